// Library-internal declarations shared by the host API and the kernels of
// libssp.  Not part of the public ABI (include/ssp.h is).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ssp {

constexpr int kWaveSize = 64;
constexpr int kWavesPerGroup = 4;
constexpr int kGroupThreads = kWaveSize * kWavesPerGroup;
constexpr int kMaxBeads = 128;
constexpr int kSampleValues = 12;  // sigma (6) then sigma^v (6)
constexpr int kCorrLags = 16;
constexpr int kMaxCorrLevels = 16;
// Chains the allocation-free reverse pass can reduce (its static scratch holds
// 10 FP64 gradients per chain: 20 MiB per GPU).
constexpr int64_t kNoAllocMaxChains = int64_t(1) << 18;

// ctrl[] words in the work buffer (device-resident so that captured graphs
// can be replayed at any step count).
enum CtrlWord { kCtrlSteps = 0, kCtrlCorrSamples = 1, kCtrlSeriesSamples = 2, kCtrlWords = 8 };
enum FlagBits { kFlagNonFinite = 1u, kFlagSeriesOverflow = 2u, kFlagInternal = 4u, kFlagReplay = 8u, kFlagLogOverflow = 16u };

// Random-stream purposes (last counter word = step hi | purpose << 24).
enum Purpose : uint32_t {
    kInitBond = 1,
    kInitZ = 2,
    kInitS = 3,
    kInitAnchor = 4,
    kNoise = 5,
    kSlot = 6,
    kAnchor = 7,
    kNoise2 = 8
};

struct ChainTables {
    const int64_t* off;   // [M] first bead / slot entry of the chain
    const int32_t* n;     // [M] beads (= slots)
    const int32_t* elem;  // [M] element of the chain
    const uint32_t* gid;  // [M] global chain id (random-stream key)
};

// Canonical device state.  FP32: r0 = R hi, r1 = R lo, a0 = A hi, a1 = A lo
// (float4, w unused).  FP64: r0 = R, a0 = A (double4, w unused); r1, a1 null.
struct State {
    void* r0;
    void* r1;
    void* a0;
    void* a1;
    int32_t* s;
};

struct Physics {
    double dt, n0, ns, zeta_s;
    uint32_t key0, key1;
};

struct StepArgs {
    State st;  // read at launch start, written back at the end (a replay only reads it)
    ChainTables ct;
    const int32_t* tasks;  // chains handled by this launch, one per segment
    int64_t n_tasks;
    const double* kappa;   // [E][9]
    const uint32_t* thr;   // [2][kMaxBeads+1]: integer thresholds for p_K and 2 p_K
    uint32_t thr_destroy;
    int32_t construct_rule;  // 0: K = C - Z attempts; 1: K = 1, the lowest empty slot attempts
    Physics ph;
    const int64_t* ctrl;
    int32_t n_steps;
    int32_t sample_every;  // 0: no sampling
    double* samples;       // [Qcap][M][12] or null
    int64_t n_chains;
    uint32_t* flags;
    // adjoint support (all optional)
    int8_t* rec_s;         // [window+1][total]: slot state after step g stored at row g + 1 - rec_g0
    State ck_end;          // optional (r0 null: off): a second copy of the final state, in the state-buffer layout
    int64_t rec_g0;
    const int8_t* replay_s;  // [window+1][total], rows as rec_s: replay these slot states instead of deciding them
    int64_t total;         // beads (= slots) in the ensemble
    // Trajectory output.  Replay (with replay_s), rows 0..n_steps of the launch:
    //   traj  [n_steps+1][total] T3: R at launch start and after every step;
    //   traj2 [n_steps+1][total] T3: A of every slot at row n_steps; at row m + 1 the anchor of each
    //         spring destroyed in step m (as advected by that step); nothing else.
    // Storing forward (traj set, no replay_s), rows counted from the window start (rec_g0):
    //   traj  [window+1][total] T3: R as above;
    //   traj2 [total] T3: A of every slot at the end of the launch;
    //   dlog  [chains][dcap] T3: per chain, the anchor of each destroyed spring, in step order and
    //         within a step in slot order (the same for every mapping); dcnt [chains]: entries so
    //         far (a count above dcap means the excess was not written).
    void* traj;
    void* traj2;
    void* dlog;
    int64_t* dcnt;
    // Persistent schedule (plain step launches only; null: one wavefront per
    // wave task for the whole launch): sched[0] the unit counter, sched[1 +
    // w] the chunks of wave task w finished, all zero at launch; chunk: steps
    // per unit; n_wave_tasks: wavefronts' worth of tasks.
    uint32_t* sched;
    int32_t chunk;
    int64_t n_wave_tasks;
    int32_t dcap;
};

struct AdjointArgs {
    ChainTables ct;
    const int32_t* tasks;
    int64_t n_tasks;
    const double* kappa;    // [E][9]
    Physics ph;
    const int8_t* rec_s;    // [window+1][total]
    int64_t rec_g0;         // global step index of the window start
    int64_t m0;             // window index of the segment start
    int32_t len;            // steps in the segment
    const void* traj;       // [len+1][total] T3: R (replay or storing-forward output)
    const void* traj2;      // replay: [len+1][total] T3, A at row len and of the springs destroyed in each
                            // step; stored window: [total] T3, A at the window end
    const void* dlog;       // stored window: destroyed-spring anchors per chain (as StepArgs)
    const int64_t* dcnt;    // stored window: log entries per chain
    int32_t dcap;
    void* lam;              // [total][6] T: dJ/dR, dJ/dA carried between segments
    double* grad;           // [M][10]: dJ/dkappa (row-major), dJ/dN_s (accumulated)
    uint32_t* flags;        // kFlagReplay: a recorded slot row out of range (read as empty), an impossible
                            // move, or a destruction log that does not match the rows; kFlagLogOverflow
    int64_t total;
    int32_t comp;           // objective component 0..5 (xx yy zz xy yz zx)
    int32_t seed_lambda;    // 1 for the last segment: start from dJ/dR at its end
    int32_t init_terms;     // 1: include the N_s dependence of the sampled initial anchors (segment at window start)
    int32_t stored;         // 1: a stored window (no replay has checked its rows; anchors from dlog)
};

struct CorrArgs {
    const double* samples;  // [Qcap][M][12]
    double* hist;           // [L][3M][16] lag history of y at each level
    double* acc;            // [L][3M][16] accumulated x(t) y(t - k)
    double* pend;           // [3M][16][2] pending (x, y) of level = lane
    double* acc_v;          // [L][3M][16] accumulated x_v(t) y(t - k), x_v = sigma^v (or null: channel off)
    double* pend_v;         // [3M][16] pending x_v of level = lane
    int64_t n_chains;
    int32_t levels;
    int32_t n_steps;
    int32_t sample_every;
    const int64_t* ctrl;
};

// Launchers (ssp_kernels.hip).
hipError_t launch_step(int precision, int W, int B, const StepArgs& a, hipStream_t s);
hipError_t launch_init(int precision, const State& st, const ChainTables& ct, int64_t M, Physics ph,
                       hipStream_t s);
hipError_t launch_reset_ctrl(int64_t* ctrl, uint32_t* flags, hipStream_t s);
hipError_t launch_zero(double* p, int64_t count, hipStream_t s);
hipError_t launch_zero_ctrl_obs(int64_t* ctrl, hipStream_t s);
hipError_t launch_advance(int64_t* ctrl, int32_t n_steps, int32_t sample_every, int64_t series_cap,
                          uint32_t* flags, hipStream_t s);
hipError_t launch_corr(const CorrArgs& a, hipStream_t s);
hipError_t launch_corr_batches(const double* acc, int64_t n_chains, int32_t levels, int32_t batches,
                               double* out, hipStream_t s);
hipError_t launch_corr_final(const double* batch_sums, int64_t n_chains, int32_t levels, int32_t batches,
                             int64_t corr_samples, double* G, double* G_err, hipStream_t s);
hipError_t launch_series(const double* samples, const int32_t* elem_off, int32_t n_elements, int64_t n_chains,
                         int32_t n_steps, int32_t sample_every, int64_t q_cap, const int64_t* ctrl,
                         double* series, int64_t series_cap, hipStream_t s);
hipError_t launch_stress(int precision, const State& st, const ChainTables& ct, int64_t M, double ns, double* out,
                         hipStream_t s);
hipError_t launch_read_state(int precision, const State& st, int64_t total, double* R, double* A, int32_t* S,
                             hipStream_t s);
hipError_t launch_write_state(int precision, const State& st, int64_t total, const double* R, const double* A,
                              const int32_t* S, hipStream_t s);
hipError_t launch_adjoint(int precision, int W, int B, const AdjointArgs& a, hipStream_t s);
hipError_t launch_copy_bytes(void* dst, const void* src, size_t bytes, hipStream_t s);
hipError_t launch_rec_s0(const int32_t* S, int8_t* rec, int64_t total, hipStream_t s);
hipError_t launch_set_ctrl_steps(int64_t* ctrl, int64_t steps, hipStream_t s);
hipError_t launch_rng_normals(int precision, uint32_t key0, uint32_t key1, uint32_t gid, int64_t step, int32_t bead,
                              int32_t count, double* out, hipStream_t s);
// Device address of the static scratch of ssp_adjoint_elements_noalloc on
// `device`, which must be current (looked up once per device).
hipError_t noalloc_scratch(int device, double** ptr);
hipError_t launch_element_mean(const double* rows, int64_t stride, int32_t ncols, const int32_t* elem_off,
                               int32_t n_elements, double* out, hipStream_t s);
hipError_t launch_grid_ratio(const double* num, const double* den, int32_t levels, int64_t samples, double* ratio,
                             hipStream_t s);
hipError_t launch_moduli(const double* G, int32_t levels, int64_t samples, double sample_dt, const double* omega,
                         int32_t n_omega, double t_lo, double t_hi, double* moduli, double* scalars, hipStream_t s);

}  // namespace ssp
