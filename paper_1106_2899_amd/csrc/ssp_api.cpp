// Host side of libssp: configuration checks, device memory layout inside the
// caller's buffers, launch sequencing, hipGraph capture/replay, and the
// extern "C" entry points declared in include/ssp.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "../../include/ssp.h"
#include "ssp_internal.h"

using namespace ssp;

namespace {

thread_local std::string g_create_error;
thread_local std::string g_create_warning;

// Sec. 3.1 caps the hop probabilities at 1/2, the construction probability
// per attempt at 1/2 and the destruction probability at 1; at dt / zeta_s =
// 0.1 (Sec. 4.1) none of them binds.  Above dt / zeta_s = 1/4 a hop
// probability 2 (dt / zeta_s) / (1 + e^{2 q y}) can reach 1/2 for y < 0, and
// the step no longer follows the continuous-time rates it discretises: a
// configuration that large is accepted, with a warning.
std::string cap_warning(const ssp_config& k)
{
    const double h = k.dt / k.zeta_s;
    if (!(h > 0.25)) return std::string();
    char buf[256];
    std::snprintf(buf, sizeof buf,
                  "dt/zeta_s = %.4g > 0.25: the 1/2 caps on the hop probabilities%s%s bind (Sec. 3.1 step map)", h,
                  (h / k.n0 > 0.5) ? ", the construction probability" : "",
                  (h >= 1.0) ? " and the destruction probability" : "");
    return std::string(buf);
}

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Chain-to-wavefront mapping of one group of chains: segment width W lanes
// and B beads per lane, W * B >= N for every chain of the group.
struct Mapping {
    int W, B;
    bool operator<(const Mapping& o) const { return W != o.W ? W < o.W : B < o.B; }
};

Mapping default_mapping(int n)
{
    if (n <= 8) return {8, 1};
    if (n <= 16) return {16, 1};
    if (n <= 32) return {32, 1};
    if (n <= 64) return {64, 1};
    return {64, 2};
}

bool mapping_supported(int W, int B)
{
    if (B == 1) return W == 8 || W == 16 || W == 32 || W == 64;
    if (B == 2) return W == 16 || W == 32 || W == 64;
    return false;
}

struct Layout {
    // work buffer offsets (bytes)
    size_t ctrl, flags, off, n, elem, gid, tasks, elem_off, thr, samples, hist, acc, pend, acc_v, pend_v, batch,
        series, corr_out, sched, total;
    // state buffer offsets
    size_t r0, r1, a0, a1, s, state_total;
    int64_t q_cap;
    int32_t chunk;
};

struct Resolved {
    ssp_config cfg;
    std::vector<int32_t> N;
    std::vector<int32_t> elem_off;
    std::vector<int64_t> ids;
    int64_t total_beads = 0;
};

bool resolve(const ssp_config* c, Resolved& r, std::string& err)
{
    if (!c) {
        err = "null config";
        return false;
    }
    r.cfg = *c;
    const ssp_config& k = r.cfg;
    if (k.n_chains < 1) {
        err = "n_chains must be >= 1";
        return false;
    }
    if (k.n_chains > (int64_t)INT32_MAX) {
        err = "n_chains must fit in int32";
        return false;
    }
    if (k.n_elements < 1 || k.n_elements > k.n_chains) {
        err = "n_elements must be in 1..n_chains";
        return false;
    }
    if (k.precision != SSP_FP32 && k.precision != SSP_FP64) {
        err = "precision must be SSP_FP32 or SSP_FP64";
        return false;
    }
    if (!(k.dt > 0.0) || !(k.n0 > 0.0) || !(k.ns > 0.0) || !(k.zeta_s > 0.0) || !std::isfinite(k.dt) ||
        !std::isfinite(k.ns) || !std::isfinite(k.zeta_s)) {
        err = "dt, n0, ns and zeta_s must be positive and finite";
        return false;
    }
    if (k.sample_every < 1) {
        err = "sample_every must be >= 1";
        return false;
    }
    if (k.corr_levels < 0 || k.corr_levels > kMaxCorrLevels) {
        err = "corr_levels must be in 0..16";
        return false;
    }
    if (k.corr_levels > 0 && k.corr_lags != kCorrLags) {
        err = "corr_lags must be 16";
        return false;
    }
    if (k.corr_levels > 0 && (k.corr_batches < 1 || k.corr_batches > 64 || k.corr_batches > k.n_chains)) {
        err = "corr_batches must be in 1..min(64, n_chains)";
        return false;
    }
    if (k.series_capacity < 0) {
        err = "series_capacity must be >= 0";
        return false;
    }
    if (k.max_steps_per_launch < 0) {
        err = "max_steps_per_launch must be >= 0";
        return false;
    }
    if (k.construct_rule != 0 && k.construct_rule != 1) {
        err = "construct_rule must be 0 (K = C - Z) or 1 (K = 1)";
        return false;
    }
    if (k.corr_virtual != 0 && k.corr_virtual != 1) {
        err = "corr_virtual must be 0 or 1";
        return false;
    }
    const int64_t M = k.n_chains;
    r.N.resize(M);
    for (int64_t i = 0; i < M; ++i) {
        const int32_t n = k.n_beads_host ? k.n_beads_host[i] : k.n_beads;
        if (n < 2 || n > SSP_MAX_BEADS) {
            err = "every chain needs 2 <= N <= 128 beads (chain " + std::to_string(i) + ")";
            return false;
        }
        r.N[i] = n;
        r.total_beads += n;
    }
    r.elem_off.resize(k.n_elements + 1);
    if (k.element_offsets_host) {
        for (int e = 0; e <= k.n_elements; ++e) r.elem_off[e] = k.element_offsets_host[e];
        if (r.elem_off[0] != 0 || r.elem_off[k.n_elements] != M) {
            err = "element_offsets must start at 0 and end at n_chains";
            return false;
        }
        for (int e = 0; e < k.n_elements; ++e)
            if (r.elem_off[e + 1] <= r.elem_off[e]) {
                err = "element_offsets must be strictly increasing";
                return false;
            }
    } else {
        for (int e = 0; e <= k.n_elements; ++e) r.elem_off[e] = (int32_t)(M * e / k.n_elements);
        for (int e = 0; e < k.n_elements; ++e)
            if (r.elem_off[e + 1] <= r.elem_off[e]) {
                err = "empty element in equal split";
                return false;
            }
    }
    r.ids.resize(M);
    for (int64_t i = 0; i < M; ++i) {
        r.ids[i] = k.chain_ids_host ? k.chain_ids_host[i] : i;
        if (r.ids[i] < 0 || r.ids[i] > (int64_t)UINT32_MAX) {
            err = "chain ids must be in 0..2^32-1";
            return false;
        }
    }
    return true;
}

Layout make_layout(const Resolved& r)
{
    const ssp_config& k = r.cfg;
    const int64_t M = k.n_chains;
    Layout L{};
    // steps per launch: bounded so that the per-launch sample buffer stays below
    // about 1 GiB (12 FP64 values per chain and sample).
    int32_t chunk = k.max_steps_per_launch;
    if (chunk == 0) {
        const double per_sample = (double)M * kSampleValues * 8.0;
        int64_t max_q = (int64_t)std::max(1.0, std::floor((1024.0 * 1024.0 * 1024.0) / per_sample));
        int64_t c = std::min<int64_t>(1000, max_q * k.sample_every);
        chunk = (int32_t)std::max<int64_t>(1, c);
    }
    L.chunk = chunk;
    L.q_cap = chunk / k.sample_every + 1;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    L.ctrl = take(sizeof(int64_t) * kCtrlWords);
    L.flags = take(sizeof(uint32_t));
    L.off = take(sizeof(int64_t) * M);
    L.n = take(sizeof(int32_t) * M);
    L.elem = take(sizeof(int32_t) * M);
    L.gid = take(sizeof(uint32_t) * M);
    L.tasks = take(sizeof(int32_t) * M);
    L.elem_off = take(sizeof(int32_t) * (k.n_elements + 1));
    L.thr = take(sizeof(uint32_t) * 2 * (kMaxBeads + 1));
    L.samples = take(sizeof(double) * (size_t)L.q_cap * M * kSampleValues);
    const int lv = k.corr_levels;
    L.hist = take(lv ? sizeof(double) * (size_t)lv * 3 * M * 16 : 0);
    L.acc = take(lv ? sizeof(double) * (size_t)lv * 3 * M * 16 : 0);
    L.pend = take(lv ? sizeof(double) * (size_t)3 * M * 16 * 2 : 0);
    const bool cv = lv && k.corr_virtual;
    L.acc_v = take(cv ? sizeof(double) * (size_t)lv * 3 * M * 16 : 0);
    L.pend_v = take(cv ? sizeof(double) * (size_t)3 * M * 16 : 0);
    L.batch = take(lv ? sizeof(double) * (size_t)k.corr_batches * lv * 16 : 0);
    L.corr_out = take(lv ? sizeof(double) * (size_t)lv * 16 * 2 : 0);
    // persistent schedule: per mapping group a counter and a word per wave task
    // (at most M + 8 words), zeroed as (M + 17) / 2 doubles
    L.sched = take(sizeof(uint32_t) * (size_t)(M + 18));
    L.series = take(sizeof(double) * (size_t)k.n_elements * k.series_capacity * 6);
    L.total = o;
    const size_t beads = (size_t)r.total_beads;
    const size_t v4 = k.precision == SSP_FP32 ? 16 : 32;
    o = 0;
    L.r0 = take(v4 * beads);
    L.r1 = k.precision == SSP_FP32 ? take(v4 * beads) : 0;
    L.a0 = take(v4 * beads);
    L.a1 = k.precision == SSP_FP32 ? take(v4 * beads) : 0;
    L.s = take(sizeof(int32_t) * beads);
    L.state_total = o;
    return L;
}

// Integer form of u < p for u = ((w >> 9) + 1/2) 2^-23: (w >> 9) < ceil(p 2^23 - 1/2).
uint32_t threshold(double p)
{
    const double x = std::ceil(p * 8388608.0 - 0.5);
    if (x <= 0.0) return 0u;
    if (x >= 8388608.0) return 8388608u;
    return (uint32_t)x;
}

}  // namespace

struct ssp_handle {
    Resolved res;
    Layout lay;
    int device = 0;
    char* state = nullptr;
    char* work = nullptr;
    std::vector<std::pair<Mapping, std::pair<int64_t, int64_t>>> groups;  // mapping, [task begin, count)
    std::vector<Mapping> chain_map;                                       // mapping of every chain
    // last recorded window (adjoint)
    struct {
        const void* ptr = nullptr;
        int64_t window = 0, g0 = 0;
        int32_t ckpt = 0;
        bool stored = false;  // the forward stored the trajectory (one segment)
    } rec;
    bool initialized = false;
    int64_t steps = 0, corr_samples = 0, series_samples = 0;
    hipStream_t capture_stream = nullptr;
    std::map<std::pair<int64_t, const double*>, hipGraphExec_t> graphs;
    std::string err;
    std::string warning;  // set at creation (cap_warning)
    bool persistent = true;  // plain steps run the persistent schedule (ssp_set_schedule)
    // device address of the static scratch of the allocation-free reverse
    // pass, looked up at creation (null if the lookup failed; hipError kept)
    double* noalloc = nullptr;
    hipError_t noalloc_err = hipSuccess;
    // kernel timing mode: events bracket every step-kernel launch
    bool timing = false;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
    double timed_ms = 0.0;
    int64_t timed_launches = 0, timed_bead_steps = 0;

    State st() const
    {
        State s;
        s.r0 = state + lay.r0;
        s.r1 = lay.r1 ? state + lay.r1 : nullptr;
        s.a0 = state + lay.a0;
        s.a1 = lay.a1 ? state + lay.a1 : nullptr;
        if (res.cfg.precision == SSP_FP64) {
            s.r1 = nullptr;
            s.a1 = nullptr;
        }
        s.s = reinterpret_cast<int32_t*>(state + lay.s);
        return s;
    }
    ChainTables ct() const
    {
        ChainTables c;
        c.off = reinterpret_cast<const int64_t*>(work + lay.off);
        c.n = reinterpret_cast<const int32_t*>(work + lay.n);
        c.elem = reinterpret_cast<const int32_t*>(work + lay.elem);
        c.gid = reinterpret_cast<const uint32_t*>(work + lay.gid);
        return c;
    }
    int64_t* ctrl() const { return reinterpret_cast<int64_t*>(work + lay.ctrl); }
    uint32_t* flags() const { return reinterpret_cast<uint32_t*>(work + lay.flags); }
    double* samples() const { return reinterpret_cast<double*>(work + lay.samples); }
    Physics phys() const
    {
        Physics p;
        p.dt = res.cfg.dt;
        p.n0 = res.cfg.n0;
        p.ns = res.cfg.ns;
        p.zeta_s = res.cfg.zeta_s;
        p.key0 = (uint32_t)(res.cfg.seed & 0xffffffffu);
        p.key1 = (uint32_t)(res.cfg.seed >> 32);
        return p;
    }
};

namespace {

int fail(ssp_handle* h, int code, const std::string& msg)
{
    if (h) h->err = msg;
    return code;
}

#define HIPCHK(h, expr)                                                                                   \
    do {                                                                                                  \
        hipError_t e_ = (expr);                                                                           \
        if (e_ != hipSuccess) return fail((h), SSP_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ck_end (optional): where the last launch also writes the final state.
// Outputs of a storing forward (see StepArgs).
struct StoreOut {
    void* traj = nullptr;
    void* traj2 = nullptr;
    void* dlog = nullptr;
    int64_t* dcnt = nullptr;
    int32_t dcap = 0;
};

int enqueue_steps(ssp_handle* h, int64_t n, const double* kappa, hipStream_t s, int8_t* rec_s = nullptr,
                  int64_t rec_g0 = 0, const State* ck_end = nullptr, const StoreOut* out = nullptr)
{
    const ssp_config& k = h->res.cfg;
    const int64_t M = k.n_chains;
    for (int64_t done = 0; done < n;) {
        const int32_t m = (int32_t)std::min<int64_t>(h->lay.chunk, n - done);
        // a plain step (nothing recorded or stored) runs the persistent schedule
        const bool persistent = !rec_s && !ck_end && !out && h->persistent;
        uint32_t* sched = reinterpret_cast<uint32_t*>(h->work + h->lay.sched);
        if (persistent) HIPCHK(h, launch_zero(reinterpret_cast<double*>(sched), (M + 16 + 1) / 2, s));
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (h->timing) {
            HIPCHK(h, hipEventCreate(&e0));
            HIPCHK(h, hipEventCreate(&e1));
            HIPCHK(h, hipEventRecord(e0, s));
        }
        for (auto& g : h->groups) {
            StepArgs a{};
            if (persistent) {  // each group's counter and progress words after the previous group's
                const int64_t cpw = kWaveSize / g.first.W;
                a.n_wave_tasks = (g.second.second + cpw - 1) / cpw;
                a.sched = sched;
                sched += 1 + a.n_wave_tasks;
                a.chunk = m;  // the launcher picks the chunk length
            }
            a.st = h->st();
            a.ct = h->ct();
            a.tasks = reinterpret_cast<const int32_t*>(h->work + h->lay.tasks) + g.second.first;
            a.n_tasks = g.second.second;
            a.kappa = kappa;
            a.thr = reinterpret_cast<const uint32_t*>(h->work + h->lay.thr);
            a.thr_destroy = threshold(std::min(k.dt / k.zeta_s * 1.0, 1.0));
            a.construct_rule = k.construct_rule;
            a.ph = h->phys();
            a.ctrl = h->ctrl();
            a.n_steps = m;
            a.sample_every = k.sample_every;
            a.samples = h->samples();
            a.n_chains = M;
            a.flags = h->flags();
            a.rec_s = rec_s;
            a.rec_g0 = rec_g0;
            if (ck_end && done + m == n) a.ck_end = *ck_end;
            if (out) {
                a.traj = out->traj;
                a.traj2 = out->traj2;
                a.dlog = out->dlog;
                a.dcnt = out->dcnt;
                a.dcap = out->dcap;
            }
            a.total = h->res.total_beads;
            HIPCHK(h, launch_step(k.precision, g.first.W, g.first.B, a, s));
        }
        if (h->timing) {
            HIPCHK(h, hipEventRecord(e1, s));
            h->events.push_back({e0, e1});
            h->timed_bead_steps += h->res.total_beads * (int64_t)m;
        }
        if (k.corr_levels > 0) {
            CorrArgs c{};
            c.samples = h->samples();
            c.hist = reinterpret_cast<double*>(h->work + h->lay.hist);
            c.acc = reinterpret_cast<double*>(h->work + h->lay.acc);
            c.pend = reinterpret_cast<double*>(h->work + h->lay.pend);
            if (k.corr_virtual) {
                c.acc_v = reinterpret_cast<double*>(h->work + h->lay.acc_v);
                c.pend_v = reinterpret_cast<double*>(h->work + h->lay.pend_v);
            }
            c.n_chains = M;
            c.levels = k.corr_levels;
            c.n_steps = m;
            c.sample_every = k.sample_every;
            c.ctrl = h->ctrl();
            HIPCHK(h, launch_corr(c, s));
        }
        if (k.series_capacity > 0) {
            HIPCHK(h, launch_series(h->samples(), reinterpret_cast<const int32_t*>(h->work + h->lay.elem_off),
                                    k.n_elements, M, m, k.sample_every, h->lay.q_cap, h->ctrl(),
                                    reinterpret_cast<double*>(h->work + h->lay.series), k.series_capacity, s));
        }
        HIPCHK(h, launch_advance(h->ctrl(), m, k.sample_every, k.series_capacity, h->flags(), s));
        done += m;
    }
    return SSP_OK;
}

int64_t samples_between(int64_t g0, int64_t n, int32_t every) { return (g0 + n) / every - g0 / every; }

// Groups chains by their mapping (chain order kept inside a group) and
// returns the concatenated task list; h->groups receives the ranges.
std::vector<int32_t> group_tasks(ssp_handle* h)
{
    std::map<Mapping, std::vector<int32_t>> by;
    for (size_t i = 0; i < h->chain_map.size(); ++i) by[h->chain_map[i]].push_back((int32_t)i);
    std::vector<int32_t> tasks;
    tasks.reserve(h->chain_map.size());
    h->groups.clear();
    for (auto& kv : by) {
        h->groups.push_back({kv.first, {(int64_t)tasks.size(), (int64_t)kv.second.size()}});
        tasks.insert(tasks.end(), kv.second.begin(), kv.second.end());
    }
    return tasks;
}

int check_flags(ssp_handle* h, hipStream_t s)
{
    uint32_t f = 0;
    HIPCHK(h, hipMemcpyAsync(&f, h->flags(), sizeof(f), hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    if (f & kFlagNonFinite) return fail(h, SSP_ENONFINITE, "a non-finite bead position was produced");
    if (f & kFlagInternal) return fail(h, SSP_EHIP, "internal error: slip-spring force gather did not complete");
    return SSP_OK;
}

int zero_observables(ssp_handle* h, hipStream_t s)
{
    const ssp_config& k = h->res.cfg;
    const int64_t M = k.n_chains;
    if (k.corr_levels > 0) {
        HIPCHK(h, launch_zero(reinterpret_cast<double*>(h->work + h->lay.hist), (int64_t)k.corr_levels * 3 * M * 16, s));
        HIPCHK(h, launch_zero(reinterpret_cast<double*>(h->work + h->lay.acc), (int64_t)k.corr_levels * 3 * M * 16, s));
        HIPCHK(h, launch_zero(reinterpret_cast<double*>(h->work + h->lay.pend), 3 * M * 16 * 2, s));
        if (k.corr_virtual) {
            HIPCHK(h, launch_zero(reinterpret_cast<double*>(h->work + h->lay.acc_v), (int64_t)k.corr_levels * 3 * M * 16, s));
            HIPCHK(h, launch_zero(reinterpret_cast<double*>(h->work + h->lay.pend_v), 3 * M * 16, s));
        }
    }
    if (k.series_capacity > 0)
        HIPCHK(h, launch_zero(reinterpret_cast<double*>(h->work + h->lay.series),
                              (int64_t)k.n_elements * k.series_capacity * 6, s));
    HIPCHK(h, launch_zero_ctrl_obs(h->ctrl(), s));
    h->corr_samples = 0;
    h->series_samples = 0;
    return SSP_OK;
}

}  // namespace

extern "C" {

int ssp_config_init(ssp_config* c)
{
    if (!c) return SSP_EINVAL;
    std::memset(c, 0, sizeof(*c));
    c->n_chains = 1;
    c->n_elements = 1;
    c->precision = SSP_FP32;
    c->n_beads = 8;
    c->sample_every = 1;
    c->dt = 0.01;
    c->n0 = 4.0;
    c->ns = 0.5;
    c->zeta_s = 0.1;
    c->seed = 1;
    c->corr_levels = 16;
    c->corr_lags = 16;
    c->corr_batches = 16;
    c->series_capacity = 0;
    c->use_graph = 1;
    c->construct_rule = 0;
    c->corr_virtual = 0;
    return SSP_OK;
}

int ssp_query_sizes(const ssp_config* cfg, size_t* state_bytes, size_t* work_bytes)
{
    Resolved r;
    g_create_warning.clear();
    if (!resolve(cfg, r, g_create_error)) return SSP_EINVAL;
    g_create_warning = cap_warning(r.cfg);
    if (cfg->corr_levels > 0 && cfg->corr_batches > cfg->n_chains) {
        g_create_error = "corr_batches exceeds n_chains";
        return SSP_EINVAL;
    }
    const Layout L = make_layout(r);
    if (state_bytes) *state_bytes = L.state_total;
    if (work_bytes) *work_bytes = L.total;
    return SSP_OK;
}

int ssp_create(const ssp_config* cfg, void* state_dev, void* work_dev, ssp_handle** out)
{
    if (!out) {
        g_create_error = "null output handle";
        return SSP_EINVAL;
    }
    *out = nullptr;
    if (!state_dev || !work_dev) {
        g_create_error = "state and work buffers are required";
        return SSP_EINVAL;
    }
    if ((reinterpret_cast<uintptr_t>(state_dev) % kAlign) || (reinterpret_cast<uintptr_t>(work_dev) % kAlign)) {
        g_create_error = "state and work buffers must be 256-byte aligned";
        return SSP_EINVAL;
    }
    ssp_handle* h = new (std::nothrow) ssp_handle();
    if (!h) {
        g_create_error = "out of host memory";
        return SSP_EINVAL;
    }
    if (!resolve(cfg, h->res, g_create_error)) {
        delete h;
        return SSP_EINVAL;
    }
    h->warning = cap_warning(h->res.cfg);
    g_create_warning = h->warning;
    h->res.cfg.n_beads_host = nullptr;
    h->res.cfg.element_offsets_host = nullptr;
    h->res.cfg.chain_ids_host = nullptr;
    h->lay = make_layout(h->res);
    h->state = static_cast<char*>(state_dev);
    h->work = static_cast<char*>(work_dev);
    if (hipGetDevice(&h->device) != hipSuccess) {
        g_create_error = "hipGetDevice failed";
        delete h;
        return SSP_EHIP;
    }
    h->noalloc_err = noalloc_scratch(h->device, &h->noalloc);
    const int64_t M = h->res.cfg.n_chains;
    // host tables
    std::vector<int64_t> off(M);
    std::vector<int32_t> elem(M);
    std::vector<uint32_t> gid(M);
    int64_t o = 0;
    for (int64_t i = 0; i < M; ++i) {
        off[i] = o;
        o += h->res.N[i];
        gid[i] = (uint32_t)h->res.ids[i];
    }
    for (int e = 0; e < h->res.cfg.n_elements; ++e)
        for (int64_t i = h->res.elem_off[e]; i < h->res.elem_off[e + 1]; ++i) elem[i] = e;
    h->chain_map.resize(M);
    for (int64_t i = 0; i < M; ++i) h->chain_map[i] = default_mapping(h->res.N[i]);
    const std::vector<int32_t> tasks = group_tasks(h);
    std::vector<uint32_t> thr(2 * (kMaxBeads + 1), 0u);
    const ssp_config& k = h->res.cfg;
    for (int K = 1; K <= kMaxBeads; ++K) {
        double p = k.dt / (k.zeta_s * k.n0 * (double)K);
        if (p > 0.5) p = 0.5;
        thr[K] = threshold(p);
        thr[kMaxBeads + 1 + K] = threshold(2.0 * p);
    }
    auto up = [&](size_t at, const void* src, size_t bytes) {
        return hipMemcpy(h->work + at, src, bytes, hipMemcpyHostToDevice);
    };
    if (up(h->lay.off, off.data(), sizeof(int64_t) * M) != hipSuccess ||
        up(h->lay.n, h->res.N.data(), sizeof(int32_t) * M) != hipSuccess ||
        up(h->lay.elem, elem.data(), sizeof(int32_t) * M) != hipSuccess ||
        up(h->lay.gid, gid.data(), sizeof(uint32_t) * M) != hipSuccess ||
        up(h->lay.tasks, tasks.data(), sizeof(int32_t) * M) != hipSuccess ||
        up(h->lay.elem_off, h->res.elem_off.data(), sizeof(int32_t) * h->res.elem_off.size()) != hipSuccess ||
        up(h->lay.thr, thr.data(), sizeof(uint32_t) * thr.size()) != hipSuccess) {
        g_create_error = "copying the chain tables to the device failed";
        delete h;
        return SSP_EHIP;
    }
    if (hipStreamCreateWithFlags(&h->capture_stream, hipStreamNonBlocking) != hipSuccess) {
        g_create_error = "hipStreamCreateWithFlags failed";
        delete h;
        return SSP_EHIP;
    }
    *out = h;
    return SSP_OK;
}

int ssp_init_equilibrium(ssp_handle* h, ssp_stream stream)
{
    if (!h) return SSP_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIPCHK(h, hipSetDevice(h->device));
    HIPCHK(h, launch_reset_ctrl(h->ctrl(), h->flags(), s));
    HIPCHK(h, launch_init(h->res.cfg.precision, h->st(), h->ct(), h->res.cfg.n_chains, h->phys(), s));
    int rc = zero_observables(h, s);
    if (rc) return rc;
    h->steps = 0;
    h->initialized = true;
    return SSP_OK;
}

int ssp_step(ssp_handle* h, int64_t n_steps, const double* kappa_dev, ssp_stream stream)
{
    if (!h) return SSP_EINVAL;
    if (!h->initialized) return fail(h, SSP_ESTATE, "ssp_step before ssp_init_equilibrium");
    if (n_steps < 0) return fail(h, SSP_EINVAL, "n_steps must be >= 0");
    if (n_steps == 0) return SSP_OK;
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIPCHK(h, hipSetDevice(h->device));
    if (h->res.cfg.use_graph && !h->timing) {
        const auto key = std::make_pair(n_steps, kappa_dev);
        auto it = h->graphs.find(key);
        if (it == h->graphs.end()) {
            hipGraph_t graph = nullptr;
            HIPCHK(h, hipStreamBeginCapture(h->capture_stream, hipStreamCaptureModeRelaxed));
            int rc = enqueue_steps(h, n_steps, kappa_dev, h->capture_stream);
            hipError_t ec = hipStreamEndCapture(h->capture_stream, &graph);
            if (rc) return rc;
            if (ec != hipSuccess) return fail(h, SSP_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(ec));
            hipGraphExec_t exec = nullptr;
            ec = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ec != hipSuccess) return fail(h, SSP_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(ec));
            it = h->graphs.emplace(key, exec).first;
        }
        HIPCHK(h, hipGraphLaunch(it->second, s));
    } else {
        int rc = enqueue_steps(h, n_steps, kappa_dev, s);
        if (rc) return rc;
    }
    const int64_t q = samples_between(h->steps, n_steps, h->res.cfg.sample_every);
    h->steps += n_steps;
    h->corr_samples += q;
    h->series_samples += q;
    return SSP_OK;
}

int ssp_read_stress(ssp_handle* h, double* out_dev, ssp_stream stream)
{
    if (!h) return SSP_EINVAL;
    if (!h->initialized) return fail(h, SSP_ESTATE, "read before ssp_init_equilibrium");
    if (!out_dev) return fail(h, SSP_EINVAL, "out_dev is required");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIPCHK(h, hipSetDevice(h->device));
    HIPCHK(h, launch_stress(h->res.cfg.precision, h->st(), h->ct(), h->res.cfg.n_chains, h->res.cfg.ns, out_dev, s));
    return check_flags(h, s);
}

int ssp_read_element_stress(ssp_handle* h, double* out_dev, ssp_stream stream)
{
    if (!h) return SSP_EINVAL;
    if (!h->initialized) return fail(h, SSP_ESTATE, "read before ssp_init_equilibrium");
    if (!out_dev) return fail(h, SSP_EINVAL, "out_dev is required");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIPCHK(h, hipSetDevice(h->device));
    const ssp_config& k = h->res.cfg;
    // per-chain stress staged in the sample buffer, which holds at least one
    // sample of every chain and is free between steps (a launch's samples are
    // consumed by the correlator and series kernels queued right after it)
    double* per_chain = h->samples();
    HIPCHK(h, launch_stress(k.precision, h->st(), h->ct(), k.n_chains, k.ns, per_chain, s));
    HIPCHK(h, launch_element_mean(per_chain, kSampleValues, kSampleValues,
                                  reinterpret_cast<const int32_t*>(h->work + h->lay.elem_off), k.n_elements, out_dev, s));
    return check_flags(h, s);
}

int ssp_read_state(ssp_handle* h, double* R_dev, double* A_dev, int32_t* S_dev, ssp_stream stream)
{
    if (!h) return SSP_EINVAL;
    if (!R_dev || !A_dev || !S_dev) return fail(h, SSP_EINVAL, "R_dev, A_dev and S_dev are required");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIPCHK(h, hipSetDevice(h->device));
    HIPCHK(h, launch_read_state(h->res.cfg.precision, h->st(), h->res.total_beads, R_dev, A_dev, S_dev, s));
    return check_flags(h, s);
}

int ssp_write_state(ssp_handle* h, const double* R_dev, const double* A_dev, const int32_t* S_dev, ssp_stream stream)
{
    if (!h) return SSP_EINVAL;
    if (!R_dev || !A_dev || !S_dev) return fail(h, SSP_EINVAL, "R_dev, A_dev and S_dev are required");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIPCHK(h, hipSetDevice(h->device));
    // validate S on the host: it must name a bead of its own chain or be -1
    std::vector<int32_t> S(h->res.total_beads);
    HIPCHK(h, hipMemcpyAsync(S.data(), S_dev, sizeof(int32_t) * S.size(), hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    int64_t o = 0;
    for (int64_t c = 0; c < h->res.cfg.n_chains; ++c) {
        const int n = h->res.N[c];
        for (int j = 0; j < n; ++j)
            if (S[o + j] < -1 || S[o + j] >= n) return fail(h, SSP_EINVAL, "S out of range in chain " + std::to_string(c));
        o += n;
    }
    if (!h->initialized) {
        HIPCHK(h, launch_reset_ctrl(h->ctrl(), h->flags(), s));
        int rc = zero_observables(h, s);
        if (rc) return rc;
        h->steps = 0;
    }
    HIPCHK(h, launch_write_state(h->res.cfg.precision, h->st(), h->res.total_beads, R_dev, A_dev, S_dev, s));
    h->initialized = true;
    return SSP_OK;
}

int ssp_read_element_series(ssp_handle* h, double* out_dev, int64_t* n_samples_host, ssp_stream stream)
{
    if (!h) return SSP_EINVAL;
    const ssp_config& k = h->res.cfg;
    if (k.series_capacity == 0) return fail(h, SSP_ESTATE, "element series disabled (series_capacity = 0)");
    if (!out_dev) return fail(h, SSP_EINVAL, "out_dev is required");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIPCHK(h, hipSetDevice(h->device));
    HIPCHK(h, hipMemcpyAsync(out_dev, h->work + h->lay.series, sizeof(double) * k.n_elements * k.series_capacity * 6,
                             hipMemcpyDeviceToDevice, s));
    if (n_samples_host) *n_samples_host = std::min(h->series_samples, k.series_capacity);
    return check_flags(h, s);
}

int ssp_read_correlator(ssp_handle* h, double* G_dev, double* G_err_dev, double* tau_host, int64_t* counts_host,
                        ssp_stream stream)
{
    if (!h) return SSP_EINVAL;
    const ssp_config& k = h->res.cfg;
    if (k.corr_levels == 0) return fail(h, SSP_ESTATE, "correlator disabled (corr_levels = 0)");
    if (!G_dev || !G_err_dev) return fail(h, SSP_EINVAL, "G_dev and G_err_dev are required");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIPCHK(h, hipSetDevice(h->device));
    double* batch = reinterpret_cast<double*>(h->work + h->lay.batch);
    HIPCHK(h, launch_corr_batches(reinterpret_cast<const double*>(h->work + h->lay.acc), k.n_chains, k.corr_levels,
                                  k.corr_batches, batch, s));
    HIPCHK(h, launch_corr_final(batch, k.n_chains, k.corr_levels, k.corr_batches, h->corr_samples, G_dev, G_err_dev, s));
    for (int l = 0; l < k.corr_levels; ++l)
        for (int q = 0; q < 16; ++q) {
            const int64_t len = h->corr_samples >> l;
            if (tau_host) tau_host[l * 16 + q] = (double)q * std::ldexp(1.0, l) * k.sample_every * k.dt;
            if (counts_host) counts_host[l * 16 + q] = len > q ? len - q : 0;
        }
    return check_flags(h, s);
}

int ssp_read_correlator_virtual(ssp_handle* h, double* Gv_dev, double* Gv_err_dev, double* dGv_dev, ssp_stream stream)
{
    if (!h) return SSP_EINVAL;
    const ssp_config& k = h->res.cfg;
    if (k.corr_levels == 0 || !k.corr_virtual)
        return fail(h, SSP_ESTATE, "virtual-stress correlator disabled (corr_levels = 0 or corr_virtual = 0)");
    if (!Gv_dev || !Gv_err_dev) return fail(h, SSP_EINVAL, "Gv_dev and Gv_err_dev are required");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIPCHK(h, hipSetDevice(h->device));
    double* batch = reinterpret_cast<double*>(h->work + h->lay.batch);
    HIPCHK(h, launch_corr_batches(reinterpret_cast<const double*>(h->work + h->lay.acc_v), k.n_chains, k.corr_levels,
                                  k.corr_batches, batch, s));
    HIPCHK(h, launch_corr_final(batch, k.n_chains, k.corr_levels, k.corr_batches, h->corr_samples, Gv_dev, Gv_err_dev,
                                s));
    if (dGv_dev) {
        // G(t) of the same samples into the handle's own output area, then Gv / G
        double* G = reinterpret_cast<double*>(h->work + h->lay.corr_out);
        HIPCHK(h, launch_corr_batches(reinterpret_cast<const double*>(h->work + h->lay.acc), k.n_chains, k.corr_levels,
                                      k.corr_batches, batch, s));
        HIPCHK(h, launch_corr_final(batch, k.n_chains, k.corr_levels, k.corr_batches, h->corr_samples, G,
                                    G + (size_t)k.corr_levels * 16, s));
        HIPCHK(h, launch_grid_ratio(Gv_dev, G, k.corr_levels, h->corr_samples, dGv_dev, s));
    }
    return check_flags(h, s);
}

int ssp_linear_viscoelasticity(ssp_handle* h, const double* G_dev, const double* omega_dev, int32_t n_omega,
                               double t_lo, double t_hi, double* moduli_dev, double* scalars_dev, ssp_stream stream)
{
    if (!h) return SSP_EINVAL;
    const ssp_config& k = h->res.cfg;
    if (k.corr_levels == 0) return fail(h, SSP_ESTATE, "correlator disabled (corr_levels = 0)");
    if (!G_dev || !scalars_dev) return fail(h, SSP_EINVAL, "G_dev and scalars_dev are required");
    if (n_omega < 0) return fail(h, SSP_EINVAL, "n_omega must be >= 0");
    if (n_omega > 0 && (!omega_dev || !moduli_dev)) return fail(h, SSP_EINVAL, "omega_dev and moduli_dev are required");
    if (!(t_lo <= t_hi)) return fail(h, SSP_EINVAL, "t_lo must not exceed t_hi");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIPCHK(h, hipSetDevice(h->device));
    HIPCHK(h, launch_moduli(G_dev, k.corr_levels, h->corr_samples, k.sample_every * k.dt, omega_dev, n_omega, t_lo, t_hi,
                            moduli_dev, scalars_dev, s));
    return SSP_OK;
}

int ssp_reset_observables(ssp_handle* h, ssp_stream stream)
{
    if (!h) return SSP_EINVAL;
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIPCHK(h, hipSetDevice(h->device));
    return zero_observables(h, s);
}

int ssp_step_count(const ssp_handle* h, int64_t* steps_host)
{
    if (!h || !steps_host) return SSP_EINVAL;
    *steps_host = h->steps;
    return SSP_OK;
}

int ssp_rng_normals(ssp_handle* h, int64_t chain_id, int64_t step, int32_t bead, int32_t count, double* out_dev,
                    ssp_stream stream)
{
    if (!h) return SSP_EINVAL;
    if (!out_dev || count < 0 || bead < 0 || bead + (int64_t)count > 65536 || chain_id < 0 ||
        chain_id > (int64_t)UINT32_MAX || step < 0)
        return fail(h, SSP_EINVAL, "invalid ssp_rng_normals arguments");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIPCHK(h, hipSetDevice(h->device));
    const Physics p = h->phys();
    HIPCHK(h, launch_rng_normals(h->res.cfg.precision, p.key0, p.key1, (uint32_t)chain_id, step, bead, count, out_dev, s));
    return SSP_OK;
}

}  // extern "C"

namespace {

// Regions of a recording buffer: slot rows, checkpoints, replay state and
// control words, segment trajectory, carried adjoint.
struct RecLayout {
    size_t rows, ckpts, ctrl, traj, traj2, dlog, dcnt, lam, total;
    int n_seg;
    int32_t dcap;  // stored window: destruction-log entries per chain
};

// Destruction-log capacity per chain for a stored window.  Destructions are
// at most the initial springs (<= N) plus the creations; creations per step
// have mean K 2 p_K <= 2 dt/(zeta_s N0) under either construction rule (each
// of K attempts creates with probability 2 p_K, p_K = min{dt/(zeta_s N0 K),
// 1/2}; or K attempts when p_K is clamped, K < 2 dt/(zeta_s N0)).  The
// capacity adds 8 standard deviations of a Poisson count of that mean, plus
// 16; a chain that still overflows is reported by ssp_adjoint.
int32_t destruction_log_capacity(const ssp_handle* h, int64_t window)
{
    const ssp_config& k = h->res.cfg;
    const double mean = (double)window * 2.0 * k.dt / (k.zeta_s * k.n0);
    int32_t nmax = 0;
    for (int32_t v : h->res.N) nmax = std::max(nmax, v);
    const double cap = nmax + std::ceil(mean + 8.0 * std::sqrt(mean)) + 16.0;
    return (int32_t)std::min(cap, 1.0e9);
}

RecLayout rec_layout(const ssp_handle* h, int64_t window, int32_t ckpt)
{
    RecLayout L{};
    const size_t beads = (size_t)h->res.total_beads;
    const size_t t = h->res.cfg.precision == SSP_FP32 ? 4 : 8;
    L.n_seg = (int)((window + ckpt - 1) / ckpt);
    const size_t seg = (size_t)std::min<int64_t>(ckpt, window);  // steps of the longest segment
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    L.rows = take((size_t)(window + 1) * beads);
    L.ckpts = take((size_t)L.n_seg * h->lay.state_total);
    L.ctrl = take(sizeof(int64_t) * kCtrlWords);
    const bool store = L.n_seg == 1;  // the forward stores the window's trajectory
    L.traj = take((seg + 1) * beads * 3 * t);
    L.traj2 = take((store ? 1 : seg + 1) * beads * 3 * t);
    L.dcap = store ? destruction_log_capacity(h, window) : 0;
    L.dlog = take((size_t)h->res.cfg.n_chains * (size_t)L.dcap * 3 * t);
    L.dcnt = take(store ? sizeof(int64_t) * (size_t)h->res.cfg.n_chains : 0);
    L.lam = take(beads * 6 * t);
    L.total = o;
    return L;
}

State state_at(const ssp_handle* h, char* base)
{
    State s;
    s.r0 = base + h->lay.r0;
    s.r1 = h->res.cfg.precision == SSP_FP32 ? base + h->lay.r1 : nullptr;
    s.a0 = base + h->lay.a0;
    s.a1 = h->res.cfg.precision == SSP_FP32 ? base + h->lay.a1 : nullptr;
    s.s = reinterpret_cast<int32_t*>(base + h->lay.s);
    return s;
}

}  // namespace

extern "C" {

int ssp_adjoint_bytes(const ssp_handle* h, int64_t window, int32_t ckpt_every, size_t* bytes)
{
    if (!h || !bytes || window < 1 || ckpt_every < 1) return SSP_EINVAL;
    *bytes = rec_layout(h, window, ckpt_every).total;
    return SSP_OK;
}

int ssp_forward_record(ssp_handle* h, int64_t window, int32_t ckpt_every, const double* kappa_dev, void* rec_dev,
                       ssp_stream stream)
{
    if (!h) return SSP_EINVAL;
    if (!h->initialized) return fail(h, SSP_ESTATE, "ssp_forward_record before ssp_init_equilibrium");
    if (window < 1 || ckpt_every < 1 || !rec_dev)
        return fail(h, SSP_EINVAL, "window >= 1, ckpt_every >= 1 and rec_dev are required");
    if (reinterpret_cast<uintptr_t>(rec_dev) % kAlign) return fail(h, SSP_EINVAL, "rec_dev must be 256-byte aligned");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIPCHK(h, hipSetDevice(h->device));
    const RecLayout R = rec_layout(h, window, ckpt_every);
    char* rec = static_cast<char*>(rec_dev);
    int8_t* rows = reinterpret_cast<int8_t*>(rec + R.rows);
    const int64_t g0 = h->steps;
    HIPCHK(h, launch_rec_s0(h->st().s, rows, h->res.total_beads, s));
    // A one-segment window stores its trajectory as it runs, and the reverse
    // pass starts from that.  Otherwise checkpoint 0 is a copy of the state,
    // each segment's last launch writes the next checkpoint from its
    // epilogue, and the reverse pass replays each segment from its checkpoint.
    const bool store = R.n_seg == 1;
    StoreOut so;
    if (store) {
        so.traj = rec + R.traj;
        so.traj2 = rec + R.traj2;
        so.dlog = rec + R.dlog;
        so.dcnt = reinterpret_cast<int64_t*>(rec + R.dcnt);
        so.dcap = R.dcap;
        HIPCHK(h, launch_zero(reinterpret_cast<double*>(so.dcnt), h->res.cfg.n_chains, s));  // all-zero bits: 0
    } else {
        HIPCHK(h, launch_copy_bytes(rec + R.ckpts, h->state, h->lay.state_total, s));
    }
    h->rec.ptr = nullptr;  // not a usable recording until the window is complete
    for (int c = 0; c < R.n_seg; ++c) {
        const int64_t m = std::min<int64_t>(ckpt_every, window - (int64_t)c * ckpt_every);
        const State next = state_at(h, rec + R.ckpts + (size_t)(c + 1) * h->lay.state_total);
        int rc = enqueue_steps(h, m, kappa_dev, s, rows, g0, c + 1 < R.n_seg ? &next : nullptr,
                               store ? &so : nullptr);
        if (rc) return rc;
        const int64_t q = samples_between(h->steps, m, h->res.cfg.sample_every);
        h->steps += m;
        h->corr_samples += q;
        h->series_samples += q;
    }
    h->rec.ptr = rec_dev;
    h->rec.window = window;
    h->rec.ckpt = ckpt_every;
    h->rec.g0 = g0;
    h->rec.stored = store;
    return SSP_OK;
}

}  // extern "C"

namespace {

// The reverse pass of ssp_adjoint: per-chain gradients into grad_dev [M][10].
int adjoint_pass(ssp_handle* h, const void* rec_dev, const double* kappa_dev, int32_t component, int32_t init_window,
                 double* grad_dev, ssp_stream stream)
{
    if (!h) return SSP_EINVAL;
    if (!rec_dev || rec_dev != h->rec.ptr) return fail(h, SSP_ESTATE, "rec_dev does not hold the last recorded window");
    if (!grad_dev || component < 0 || component > 5)
        return fail(h, SSP_EINVAL, "grad_dev and component 0..5 are required");
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIPCHK(h, hipSetDevice(h->device));
    const ssp_config& k = h->res.cfg;
    const RecLayout R = rec_layout(h, h->rec.window, h->rec.ckpt);
    char* rec = static_cast<char*>(const_cast<void*>(rec_dev));
    const int8_t* rows = reinterpret_cast<const int8_t*>(rec + R.rows);
    int64_t* sctrl = reinterpret_cast<int64_t*>(rec + R.ctrl);
    HIPCHK(h, launch_zero(grad_dev, k.n_chains * 10, s));
    for (int c = R.n_seg - 1; c >= 0; --c) {
        const int64_t m = std::min<int64_t>(h->rec.ckpt, h->rec.window - (int64_t)c * h->rec.ckpt);
        // replay the segment from its checkpoint (read in place, left as it
        // is), storing the trajectory; a one-segment window has it from the
        // forward
        if (!h->rec.stored) {
            HIPCHK(h, launch_set_ctrl_steps(sctrl, h->rec.g0 + (int64_t)c * h->rec.ckpt, s));
            for (auto& g : h->groups) {
                StepArgs a{};
                a.st = state_at(h, rec + R.ckpts + (size_t)c * h->lay.state_total);  // read in place
                a.ct = h->ct();
                a.tasks = reinterpret_cast<const int32_t*>(h->work + h->lay.tasks) + g.second.first;
                a.n_tasks = g.second.second;
                a.kappa = kappa_dev;
                a.thr = reinterpret_cast<const uint32_t*>(h->work + h->lay.thr);
                a.thr_destroy = threshold(std::min(k.dt / k.zeta_s * 1.0, 1.0));
                a.construct_rule = k.construct_rule;
                a.ph = h->phys();
                a.ctrl = sctrl;
                a.n_steps = (int32_t)m;
                a.sample_every = 0;
                a.samples = nullptr;
                a.n_chains = k.n_chains;
                a.flags = h->flags();
                a.total = h->res.total_beads;
                a.traj = rec + R.traj;
                a.traj2 = rec + R.traj2;
                a.replay_s = rows;  // the recorded slot states, replayed
                a.rec_g0 = h->rec.g0;
                HIPCHK(h, launch_step(k.precision, g.first.W, g.first.B, a, s));
            }
        }
        for (auto& g : h->groups) {
            AdjointArgs a{};
            a.ct = h->ct();
            a.tasks = reinterpret_cast<const int32_t*>(h->work + h->lay.tasks) + g.second.first;
            a.n_tasks = g.second.second;
            a.kappa = kappa_dev;
            a.ph = h->phys();
            a.rec_s = rows;
            a.rec_g0 = h->rec.g0;
            a.m0 = (int64_t)c * h->rec.ckpt;
            a.len = (int32_t)m;
            a.traj = rec + R.traj;
            a.traj2 = rec + R.traj2;
            a.lam = rec + R.lam;
            a.grad = grad_dev;
            a.total = h->res.total_beads;
            a.comp = component;
            a.seed_lambda = (c == R.n_seg - 1) ? 1 : 0;
            a.init_terms = (c == 0 && init_window && h->rec.g0 == 0) ? 1 : 0;
            a.flags = h->flags();
            a.stored = h->rec.stored ? 1 : 0;  // a replay checks the rows it re-creates
            a.dlog = rec + R.dlog;
            a.dcnt = reinterpret_cast<const int64_t*>(rec + R.dcnt);
            a.dcap = R.dcap;
            HIPCHK(h, launch_adjoint(k.precision, g.first.W, g.first.B, a, s));
        }
    }
    // A bad recording leaves the ensemble itself untouched (the replay starts
    // from a checkpoint and writes only the trajectory): report it and clear
    // its flag.
    uint32_t f = 0;
    HIPCHK(h, hipMemcpyAsync(&f, h->flags(), sizeof(f), hipMemcpyDeviceToHost, s));
    HIPCHK(h, hipStreamSynchronize(s));
    if (f & kFlagLogOverflow) {
        f &= ~(uint32_t)(kFlagLogOverflow | kFlagReplay);
        HIPCHK(h, hipMemcpyAsync(h->flags(), &f, sizeof(f), hipMemcpyHostToDevice, s));
        HIPCHK(h, hipStreamSynchronize(s));
        return fail(h, SSP_ESIZE,
                    "a chain destroyed more springs in the stored window than its log holds; gradients are "
                    "invalid (record the window with checkpoints, ckpt_every < window)");
    }
    if (f & kFlagReplay) {
        f &= ~(uint32_t)kFlagReplay;
        HIPCHK(h, hipMemcpyAsync(h->flags(), &f, sizeof(f), hipMemcpyHostToDevice, s));
        HIPCHK(h, hipStreamSynchronize(s));
        return fail(h, SSP_EINVAL,
                    "the recorded slot rows are not a run of this ensemble (recording buffer changed since "
                    "ssp_forward_record, or recorded by another handle); gradients are invalid");
    }
    return check_flags(h, s);
}

}  // namespace

extern "C" {

int ssp_adjoint(ssp_handle* h, const void* rec_dev, const double* kappa_dev, int32_t component, int32_t init_window,
                double* grad_dev, ssp_stream stream)
{
    return adjoint_pass(h, rec_dev, kappa_dev, component, init_window, grad_dev, stream);
}

int ssp_adjoint_elements(ssp_handle* h, const void* rec_dev, const double* kappa_dev, int32_t component,
                         int32_t init_window, double* chain_grad_dev, double* elem_grad_dev, ssp_stream stream)
{
    if (!h) return SSP_EINVAL;
    if (!elem_grad_dev || !chain_grad_dev) return fail(h, SSP_EINVAL, "chain_grad_dev and elem_grad_dev are required");
    const int rc = adjoint_pass(h, rec_dev, kappa_dev, component, init_window, chain_grad_dev, stream);
    if (rc != SSP_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIPCHK(h, launch_element_mean(chain_grad_dev, 10, 10, reinterpret_cast<const int32_t*>(h->work + h->lay.elem_off),
                                  h->res.cfg.n_elements, elem_grad_dev, s));
    return SSP_OK;
}

int ssp_adjoint_elements_noalloc(ssp_handle* h, const void* rec_dev, const double* kappa_dev, int32_t component,
                                 int32_t init_window, double* elem_grad_dev, ssp_stream stream)
{
    if (!h) return SSP_EINVAL;
    if (!elem_grad_dev) return fail(h, SSP_EINVAL, "elem_grad_dev is required");
    if (h->res.cfg.n_chains > kNoAllocMaxChains)
        return fail(h, SSP_ESIZE, "ssp_adjoint_elements_noalloc handles at most 262144 chains (its static scratch); "
                                  "use ssp_adjoint_elements with a workspace");
    if (!h->noalloc)
        return fail(h, SSP_EHIP, std::string("the static scratch of this device is not available: ") +
                                     hipGetErrorString(h->noalloc_err));
    const int rc = adjoint_pass(h, rec_dev, kappa_dev, component, init_window, h->noalloc, stream);
    if (rc != SSP_OK) return rc;
    hipStream_t s = static_cast<hipStream_t>(stream);
    HIPCHK(h, launch_element_mean(h->noalloc, 10, 10, reinterpret_cast<const int32_t*>(h->work + h->lay.elem_off),
                                  h->res.cfg.n_elements, elem_grad_dev, s));
    return SSP_OK;
}

int ssp_set_mapping(ssp_handle* h, int32_t n_lo, int32_t n_hi, int32_t lanes_per_chain, int32_t beads_per_lane)
{
    if (!h) return SSP_EINVAL;
    if (n_lo < 2 || n_hi < n_lo || n_hi > SSP_MAX_BEADS) return fail(h, SSP_EINVAL, "need 2 <= n_lo <= n_hi <= 128");
    if (!mapping_supported(lanes_per_chain, beads_per_lane))
        return fail(h, SSP_EINVAL, "unsupported mapping (lanes 8/16/32/64 with 1 bead per lane, 16/32/64 with 2)");
    if (lanes_per_chain * beads_per_lane < n_hi)
        return fail(h, SSP_EINVAL, "lanes_per_chain * beads_per_lane must be >= n_hi");
    HIPCHK(h, hipSetDevice(h->device));
    const int64_t M = h->res.cfg.n_chains;
    for (int64_t i = 0; i < M; ++i)
        if (h->res.N[i] >= n_lo && h->res.N[i] <= n_hi) h->chain_map[i] = {lanes_per_chain, beads_per_lane};
    const std::vector<int32_t> tasks = group_tasks(h);
    HIPCHK(h, hipDeviceSynchronize());  // no launch may still read the old task list
    HIPCHK(h, hipMemcpy(h->work + h->lay.tasks, tasks.data(), sizeof(int32_t) * M, hipMemcpyHostToDevice));
    for (auto& kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
    h->graphs.clear();
    return SSP_OK;
}

int ssp_set_schedule(ssp_handle* h, int persistent)
{
    if (!h) return SSP_EINVAL;
    if ((persistent != 0) != h->persistent) {
        HIPCHK(h, hipSetDevice(h->device));
        HIPCHK(h, hipDeviceSynchronize());
        for (auto& kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
        h->graphs.clear();
        h->persistent = persistent != 0;
    }
    return SSP_OK;
}

int ssp_set_kernel_timing(ssp_handle* h, int enable)
{
    if (!h) return SSP_EINVAL;
    h->timing = enable != 0;
    return SSP_OK;
}

int ssp_kernel_time(ssp_handle* h, double* ms_host, int64_t* launches_host, int64_t* bead_steps_host)
{
    if (!h) return SSP_EINVAL;
    HIPCHK(h, hipSetDevice(h->device));
    for (auto& ev : h->events) {
        HIPCHK(h, hipEventSynchronize(ev.second));
        float ms = 0.f;
        HIPCHK(h, hipEventElapsedTime(&ms, ev.first, ev.second));
        h->timed_ms += ms;
        ++h->timed_launches;
        (void)hipEventDestroy(ev.first);
        (void)hipEventDestroy(ev.second);
    }
    h->events.clear();
    if (ms_host) *ms_host = h->timed_ms;
    if (launches_host) *launches_host = h->timed_launches;
    if (bead_steps_host) *bead_steps_host = h->timed_bead_steps;
    h->timed_ms = 0.0;
    h->timed_launches = 0;
    h->timed_bead_steps = 0;
    return SSP_OK;
}

int ssp_destroy(ssp_handle* h)
{
    if (!h) return SSP_OK;
    (void)hipSetDevice(h->device);
    for (auto& ev : h->events) {
        (void)hipEventDestroy(ev.first);
        (void)hipEventDestroy(ev.second);
    }
    for (auto& kv : h->graphs) (void)hipGraphExecDestroy(kv.second);
    if (h->capture_stream) (void)hipStreamDestroy(h->capture_stream);
    delete h;
    return SSP_OK;
}

const char* ssp_last_error(const ssp_handle* h) { return h ? h->err.c_str() : g_create_error.c_str(); }

const char* ssp_warning(const ssp_handle* h)
{
    const std::string& w = h ? h->warning : g_create_warning;
    return w.empty() ? nullptr : w.c_str();
}

}  // extern "C"
