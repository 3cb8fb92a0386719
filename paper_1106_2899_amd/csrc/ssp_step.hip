// The slip-spring ensemble step (three-substep scheme of Sec. 3.1 with the
// K = C - Z reconstruction of Sec. 3.2), one persistent launch for n steps.
//
// Mapping: a wavefront holds 64 / W chains; chain c of the wave owns the
// lane segment [W c, W c + W).  Lane li of a segment owns beads and slots
// li*B .. li*B + B - 1 (slot capacity C = N, one slot per bead).  The whole
// chain state stays in VGPRs for the n steps; it is read from HBM once at
// launch start and written once at the end.
//
// Cross-lane data paths:
//   - neighbour bonds: DPP wave shifts (VALU, no LDS traffic);
//   - per-bead records {R hi, R lo, bond right, bond left} are staged in a
//     wave-private LDS array after the move; slots read the record of their
//     bead for the hop, for new anchors and for the anchor offsets;
//   - the slot -> bead force scatter is a deterministic gather: every spring
//     sets its slot's bit in its bead's LDS mask and each bead adds the
//     offsets d of its set bits (read from LDS) in increasing slot order; no
//     float atomics, so runs are bitwise reproducible;
//   - stress sums: every lane writes its FP64 partial sums to LDS and the
//     lanes of the segment add one column each in lane order (deterministic).
//
// Per step, in the paper's order:
//   1. forces at time t: bond forces and slip-spring forces,
//   2. Euler-Maruyama move of beads and affine advection of anchors,
//   3. hops decided from the post-move positions (one uniform per spring),
//   4. destruction at the ends and K = C - Z construction attempts (integer
//      thresholds, identical in every precision),
//   5. anchor offsets recomputed from the stored positions, and the stress /
//      virtual stress of the new state every sample_every steps.
//
// k_replay is the same step with the slot decisions of 3 and 4 read from a
// recording: the adjoint's reverse pass re-creates each checkpoint segment's
// positions with it.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "ssp_device.h"
#include "ssp_internal.h"

namespace ssp {

namespace {

template <typename T> struct Vec4 {
    using type = float4;
};
template <> struct Vec4<double> {
    using type = double4;
};

template <typename T> __device__ __forceinline__ v3<T> ld3(const void* base, int64_t idx)
{
    const typename Vec4<T>::type v = reinterpret_cast<const typename Vec4<T>::type*>(base)[idx];
    return {v.x, v.y, v.z};
}
template <typename T> __device__ __forceinline__ void st3(void* base, int64_t idx, v3<T> v)
{
    typename Vec4<T>::type o;
    o.x = v.x;
    o.y = v.y;
    o.z = v.z;
    o.w = T(0);
    reinterpret_cast<typename Vec4<T>::type*>(base)[idx] = o;
}

// Per-bead record staged in LDS: R hi, R lo, bond to the right, bond from the left.
template <typename T> struct alignas(16) BeadRec {
    T v[12];
};
template <typename T> struct alignas(16) Off4 {
    T v[4];
};
template <typename T> __device__ __forceinline__ v3<T> unpack3(const Off4<T>& o) { return {o.v[0], o.v[1], o.v[2]}; }

template <typename T>
__device__ __forceinline__ void rec_put(BeadRec<T>& r, v3<T> rh, v3<T> rl, v3<T> br, v3<T> bl)
{
    BeadRec<T> t;
    t.v[0] = rh.x; t.v[1] = rh.y; t.v[2] = rh.z;
    t.v[3] = rl.x; t.v[4] = rl.y; t.v[5] = rl.z;
    t.v[6] = br.x; t.v[7] = br.y; t.v[8] = br.z;
    t.v[9] = bl.x; t.v[10] = bl.y; t.v[11] = bl.z;
    r = t;
}

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Wavefront-ordered LDS accesses of the slot masks.
template <typename M> __device__ __forceinline__ void lmask_store(M* p, M v)
{
    __hip_atomic_store(p, v, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
template <typename M> __device__ __forceinline__ M lmask_load(M* p)
{
    return __hip_atomic_load(p, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_WAVEFRONT);
}
template <typename M> __device__ __forceinline__ void lmask_or(M* p, M v)
{
    __hip_atomic_fetch_or(p, v, __ATOMIC_SEQ_CST, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

// Index of the lowest set bit, or -1 (all bits set) when there is none, as
// the hardware's find-first-bit gives it.
__device__ __forceinline__ uint32_t first_bit(uint32_t x)
{
    uint32_t r;
    asm("v_ffbl_b32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

// The slots of a segment anchored at one bead: bit j of the mask for slot j,
// in 32-bit words.
template <int kCap> struct SlotMask {
    static constexpr int kWords = (kCap + 31) / 32;
    uint32_t w[kWords];

    __device__ __forceinline__ bool any() const
    {
        uint32_t o = 0;
#pragma unroll
        for (int q = 0; q < kWords; ++q) o |= w[q];
        return o != 0;
    }
    // lowest slot in the mask, -1 when it is empty
    __device__ __forceinline__ int lowest() const
    {
        uint32_t r = first_bit(w[0]);
#pragma unroll
        for (int q = 1; q < kWords; ++q) r = min(r, first_bit(w[q]) | (32u * q));  // -1 stays -1
        return (int)r;
    }
    // removes the lowest slot
    __device__ __forceinline__ void drop()
    {
        bool below = true;  // no slot in the words below
#pragma unroll
        for (int q = 0; q < kWords; ++q) {
            const uint32_t v = w[q];
            if (q == 0)
                w[q] = v & (v - 1);  // no change when zero
            else
                w[q] = below ? (v & (v - 1)) : v;
            below = below && v == 0;
        }
    }
};

__device__ __forceinline__ bool wave_any(bool p) { return __ballot(p) != 0; }

// Ballot bits of the W-lane segment starting at lane sb.
template <int W> __device__ __forceinline__ uint64_t seg_mask(int sb)
{
    if constexpr (W == 64)
        return ~0ull;
    else
        return ((1ull << W) - 1ull) << sb;
}

template <typename T> __device__ __forceinline__ bool finite3(v3<T> v)
{
    return isfinite(v.x) && isfinite(v.y) && isfinite(v.z);
}

// Wave-private LDS: the bead records double as the transpose buffer of the
// stress sums ([64 lanes][12] FP64), which is used only after the records of
// a step have been consumed, and as the beads' slot masks of the force
// gather, which is done before the step's records are written.
// SAMP: room for the stress-sample partials (a replay samples nothing, and
// without them its LDS no longer limits the waves per SIMD).
template <typename T, int W, int B, bool SAMP> struct WaveLds {
    static constexpr int kRecBytes = (int)sizeof(BeadRec<T>) * kWaveSize * B;
    static constexpr int kSumBytes = SAMP ? (int)sizeof(double) * kWaveSize * kSampleValues : 0;
    static constexpr int kShared = kRecBytes > kSumBytes ? kRecBytes : kSumBytes;
    alignas(16) unsigned char shared[kShared];
    Off4<T> off[(kWaveSize / W) * (W * B + 1)];  // per segment: a zero entry, then the slots
    T kdt[(kWaveSize / W) * 9];                   // per segment: dt kappa (flow variants)
};

// The step, for the kernels below.  K1: construction by the K = 1 rule (one
// attempt per chain and step, by the lowest empty slot) instead of K = C - Z;
// a template parameter so that neither kernel carries the other rule's work.
// RP: replay of a recorded run: the slot state after each step is read from
// the recorded rows instead of being decided (no hop or construction draws or
// probabilities); positions and anchors follow bit for bit.
// ST: a recorded forward that also stores the trajectory the replay would
// (positions every step, the anchors the adjoint cannot rebuild), so that the
// reverse pass of a one-segment window needs no replay.  Its destroyed-spring
// anchors go to a compact per-chain log instead of a dense plane.
// FL: compiled with the flow terms (a velocity gradient table is given); a
// run at rest (no table) uses the variant without them, whose registers are
// not shared with the flow code.  The two give identical trajectories at
// kappa = 0.
template <typename T, int W, int B, bool K1, bool RP, bool ST, bool FL, bool PS>
__device__ __forceinline__ void step_body(const StepArgs& a)
{
    constexpr bool kComp = std::is_same<T, float>::value;  // (hi, lo) position sums
    constexpr int kChainsPerWave = kWaveSize / W;
    constexpr int kCap = W * B;  // bead capacity of a segment

    __shared__ WaveLds<T, W, B, !RP> lds[kWavesPerGroup];
    // creation thresholds for p_K and 2 p_K, K = 0..kMaxBeads, read every step
    __shared__ uint32_t thr[2 * (kMaxBeads + 1)];
    for (int q = threadIdx.x; q < 2 * (kMaxBeads + 1); q += kGroupThreads) thr[q] = a.thr[q];
    __syncthreads();

    const int lane = threadIdx.x & (kWaveSize - 1);
    const int wv = threadIdx.x / kWaveSize;
    const int li = lane % W;
    const int seg = lane / W;
    const int sb = lane - li;  // first lane of the segment

    // One unit of work: the chains of wave task `wtask` for n_steps steps from
    // global step g0, their samples from index q0 of the launch's sample
    // buffer on.  State is read from HBM at the start and written back at the
    // end, so units of one wave task may run on different wavefronts.
    auto run = [&](const int64_t wtask, const int64_t g0, const int32_t n_steps, const int64_t q0) {
    const int64_t task = wtask * kChainsPerWave + seg;
    const bool valid = task < a.n_tasks;
    int chain = valid ? a.tasks[task] : 0;
    int n = valid ? a.ct.n[chain] : 0;
    int64_t off = valid ? a.ct.off[chain] : 0;
    uint32_t gid = valid ? a.ct.gid[chain] : 0u;
    int elem = valid ? a.ct.elem[chain] : 0;
    if constexpr (W == kWaveSize) {
        // one chain per wavefront: its table entries go to scalar registers,
        // and the addresses built from them stay scalar
        chain = wave_uniform(chain);
        n = wave_uniform(n);
        off = wave_uniform(off);
        gid = wave_uniform(gid);
        elem = wave_uniform(elem);
    }
    BeadRec<T>* rec = reinterpret_cast<BeadRec<T>*>(lds[wv].shared);
    double* sums = reinterpret_cast<double*>(lds[wv].shared);
    const int lbase = seg * kCap;  // this segment's first entry in the LDS arrays
    // this segment's slot offsets: slot j at offs[j], a zero entry at offs[-1]
    Off4<T>* offs = lds[wv].off + seg * (kCap + 1) + 1;
    if (li == 0) offs[-1] = Off4<T>{};
    constexpr int kMaskWords = SlotMask<kCap>::kWords;
    static_assert(4 * kMaskWords <= (int)sizeof(BeadRec<T>), "the slot masks fit in the records");
    uint32_t* lmask = reinterpret_cast<uint32_t*>(lds[wv].shared);
    // word w of a bead's mask: the wavefront's words w side by side, so that
    // the lanes' accesses to their own beads fall in distinct banks
    auto mask_at = [&](int bead, int w) { return w * (kWaveSize * B) + lbase + bead; };
    uint32_t mbit[B];  // this lane's slots: their bit and word in a mask
    int mbit_word[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        mbit[b] = 1u << ((li * B + b) % 32);
        mbit_word[b] = (li * B + b) / 32;
    }

    // Step constants with dt folded in: the move is
    //   R += sqrt(2 dt) w + 3 dt (b_right - b_left) - (3/N_s) dt sum_j d_j + dt kappa R.
    const T cnoise = normal_scale<T>(sqrt(2.0 * a.ph.dt));  // Box-Muller root constant for s.d. sqrt(2 dt)
    const T cbond = T(3.0 * a.ph.dt);
    const T cspring = T(3.0 / a.ph.ns * a.ph.dt);
    const T hop_h2 = T(2.0 * a.ph.dt / a.ph.zeta_s);                    // 2 dt / zeta_s
    const T hop_e2q = glauber_exp_scale<T>(3.0 / (4.0 * a.ph.ns));     // Glauber argument scale 3/(4 N_s)
    const T asd = T(sqrt(a.ph.ns / 3.0));                               // anchor offset s.d.
    uint32_t k0 = a.ph.key0, k1 = a.ph.key1;

    T kdt_v[9];  // dt kappa of the chain's element
    uint32_t kmask = 0;  // entries of kappa that are nonzero in some chain of the wavefront
    bool chain_flow = false;  // this lane's chain has a nonzero kappa
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        kdt_v[q] = T(0);
        if constexpr (FL) {
            const double kq = valid ? a.kappa[9 * elem + q] : 0.0;
            kdt_v[q] = T(a.ph.dt * kq);
            // one chain per wavefront: its element's kappa is wave-uniform
            if constexpr (W == kWaveSize) kdt_v[q] = wave_uniform(kdt_v[q]);
            if (wave_any(kq != 0.0)) kmask |= 1u << q;
            chain_flow |= kq != 0.0;
        }
    }
    const bool flow = FL && kmask != 0;
    // elongation (a positive diagonal entry of kappa) stretches chains without
    // bound above the Rouse instability: such chains take the error-free move
    const bool chain_stretch = chain_flow && (kdt_v[0] > T(0) || kdt_v[4] > T(0) || kdt_v[8] > T(0));
    // With several chains per wavefront dt kappa differs between segments:
    // it is kept in LDS (a row per segment) and read where the flow terms use
    // it, instead of holding nine registers per lane across the steps.
    constexpr bool kKdtLds = FL && W < kWaveSize;
    T* const kdt_lds = lds[wv].kdt + seg * 9;
    if constexpr (kKdtLds) {
        if (li == 0) {
#pragma unroll
            for (int q = 0; q < 9; ++q) kdt_lds[q] = kdt_v[q];
        }
    }
    const T* kdt;
    if constexpr (kKdtLds)
        kdt = kdt_lds;
    else
        kdt = kdt_v;

    v3<T> rh[B], rl[B], ah[B], al[B], d[B], br[B], bl[B];
    int s[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int i = li * B + b;
        const bool act = i < n;
        rh[b] = act ? ld3<T>(a.st.r0, off + i) : zero3<T>();
        ah[b] = act ? ld3<T>(a.st.a0, off + i) : zero3<T>();
        if constexpr (kComp) {
            rl[b] = act ? ld3<T>(a.st.r1, off + i) : zero3<T>();
            al[b] = act ? ld3<T>(a.st.a1, off + i) : zero3<T>();
        } else {
            rl[b] = zero3<T>();
            al[b] = zero3<T>();
        }
        s[b] = act ? a.st.s[off + i] : -1;
    }

    // Bonds to the right neighbour (br) and from the left neighbour (bl) of
    // every bead owned by the lane (zero past the chain ends), then the bead
    // records in LDS.
    auto bonds_and_records = [&]() {
        const v3<T> nh = from_next3(rh[0]);
        const v3<T> nl = from_next3(rl[0]);
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int i = li * B + b;
            const v3<T> h = (b + 1 < B) ? rh[b + 1 < B ? b + 1 : b] : nh;
            const v3<T> l = (b + 1 < B) ? rl[b + 1 < B ? b + 1 : b] : nl;
            const v3<T> v = (h - rh[b]) + (l - rl[b]);  // computed everywhere, then selected
            br[b] = sel(i < n - 1, v, zero3<T>());
        }
        // The bond from the left needs no mask: the lane before the first lane
        // of a segment holds the previous segment's last bead (or is lane 0 of
        // the wave, which DPP fills with 0), and its right bond is zero since
        // it lies at or past that chain's end; past the end of this chain
        // the right bonds are zero as well.
        const v3<T> left = from_prev3(br[B - 1]);
#pragma unroll
        for (int b = 0; b < B; ++b) bl[b] = (b > 0) ? br[b > 0 ? b - 1 : 0] : left;
#pragma unroll
        for (int b = 0; b < B; ++b) rec_put(rec[lbase + li * B + b], rh[b], rl[b], br[b], bl[b]);
        wave_sync();
    };

    // Anchor offsets d_j = R_{S_j} - A_j of the occupied slots, always
    // recomputed from the stored positions (never carried across a step) so
    // that a trajectory does not depend on how steps are split into launches;
    // also staged in LDS for the next force gather.
    auto refresh_offsets = [&]() {
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int t = s[b] > 0 ? s[b] : 0;
            const BeadRec<T> r = rec[lbase + t];
            const v3<T> Rh = {r.v[0], r.v[1], r.v[2]};
            const v3<T> Rl = {r.v[3], r.v[4], r.v[5]};
            d[b] = (s[b] >= 0) ? ((Rh - ah[b]) + (Rl - al[b])) : zero3<T>();
            Off4<T> o;
            o.v[0] = d[b].x;
            o.v[1] = d[b].y;
            o.v[2] = d[b].z;
            o.v[3] = T(0);
            offs[li * B + b] = o;
        }
        wave_sync();
    };

    bonds_and_records();
    refresh_offsets();


    // Trajectory output: R after every step (row 0: the state before the
    // first step), FP32 positions rounded from hi + lo.  Anchors are written
    // only where the adjoint cannot recover them by running the advection
    // backwards: for every slot at the launch end, and for each spring
    // destroyed in a step (a replay: at that step's row; a storing forward:
    // appended to the chain's log).  A replay counts rows from its launch (one
    // segment); a storing forward from the recorded window's start, however
    // the window is split into launches.
    constexpr bool kTraj = RP || ST;
    const int64_t trow0 = RP ? 0 : g0 - a.rec_g0;
    // (the chain's row base and the lane's bead index are kept apart, so that
    // with one chain per wavefront the 64-bit part of the address is scalar)
    auto store_r = [&](int row) {
        T* base = reinterpret_cast<T*>(a.traj) + 3 * ((trow0 + row) * a.total + off);
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int i = li * B + b;
            if (i < n) {  // streamed out once, read back once by the adjoint: non-temporal
                const v3<T> v = rh[b] + rl[b];
                T* q = base + 3u * (uint32_t)i;
                __builtin_nontemporal_store(v.x, q);
                __builtin_nontemporal_store(v.y, q + 1);
                __builtin_nontemporal_store(v.z, q + 2);
            }
        }
    };
    auto store_a = [&](int row, int b) {
        v3<T>* base = reinterpret_cast<v3<T>*>(a.traj2) + ((trow0 + row) * a.total + off);
        base[(uint32_t)(li * B + b)] = ah[b] + al[b];
    };
    if constexpr (kTraj) store_r(0);
    int64_t dcount = 0;  // storing forward: entries in this chain's destruction log
    if constexpr (ST) dcount = valid ? a.dcnt[chain] : 0;
    auto log_destroyed = [&](const bool (&destroyed)[B]) {
        bool any = false;
#pragma unroll
        for (int b = 0; b < B; ++b) any |= destroyed[b];
        if (!wave_any(any)) return;
        // entries of one step in slot order (slot li B + b), whatever the mapping:
        // a slot's rank counts the destroyed slots of lower lanes and its own lower b
        const uint64_t below = (1ull << lane) - 1ull;
        int tot = 0, lower = 0;
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const uint64_t m = __ballot(destroyed[b]) & seg_mask<W>(sb);
            tot += __popcll(m);
            lower += __popcll(m & below);
        }
#pragma unroll
        for (int b = 0; b < B; ++b) {
            if (destroyed[b]) {
                const int64_t q = dcount + lower;
                if (q < a.dcap) reinterpret_cast<v3<T>*>(a.dlog)[(int64_t)chain * a.dcap + q] = ah[b] + al[b];
                ++lower;
            }
        }
        dcount += tot;
    };

    bool finite_ok = true;

    // Random streams come in step pairs (2k, 2k+1), three Philox blocks per
    // bead/slot index and pair (counter step word k):
    //   NOISE  -> Box-Muller pairs (x0,x1), (x2,x3): noise (c, s, c) of step 2k
    //             and the first normal of step 2k+1 (carried);
    //   NOISE2 -> hop / reconstruction words y2, y3 of step 2k; y0, y1 (carried)
    //             make the Box-Muller pair of the other two normals of 2k+1;
    //   SLOT   -> hop / reconstruction words z0, z1 of step 2k+1.
    // A launch that starts at an odd step rebuilds the carried values.
    T carry_n[B];
    uint32_t carry_w0[B], carry_w1[B];
#pragma unroll
    for (int b = 0; b < B; ++b) {
        carry_n[b] = T(0);
        carry_w0[b] = carry_w1[b] = 0u;
        if (g0 & 1) {
            const uint32_t i = (uint32_t)(li * B + b);
            const uint4 x = draw(kNoise, i, gid, g0 >> 1, k0, k1);
            T c;
            box_muller(x.z, x.w, cnoise, c, carry_n[b]);
            const uint4 y = draw(kNoise2, i, gid, g0 >> 1, k0, k1);
            carry_w0[b] = y.x;
            carry_w1[b] = y.y;
        }
    }
    // sampling phase: step g is sampled when (g + 1) % sample_every == 0
    int phase = a.sample_every > 0 ? (int)((g0 + 1) % a.sample_every) : 1;
    int64_t q_launch = q0;  // index in the launch's sample buffer of this unit's next sample

    // Replay: the recorded slot row of a step is loaded one step ahead, so that
    // its latency runs under the previous step.
    int replay_next[B], replay_ahead[B];
    auto replay_load = [&](int64_t gs, int (&dst)[B]) {
        const int8_t* row = a.replay_s + ((gs + 1 - a.rec_g0) * a.total + off);
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int j = li * B + b;
            dst[b] = (j < n) ? (int)row[(uint32_t)j] : -1;
        }
    };
    if constexpr (RP) {
        if (n_steps > 0) replay_load(g0, replay_ahead);
    }

    for (int step = 0; step < n_steps; ++step) {
        // the flow terms test the bits of kmask every step; recomputing those
        // tests (scalar ops) is cheaper than keeping nine hoisted conditions
        // in scalar registers across the loop, which spilled
        // Likewise the random streams' round keys (key + r x Weyl constant)
        // are recomputed by scalar adds at every draw rather than kept in
        // twenty scalar registers, which the flow variants would spill.
        if constexpr (FL) asm volatile("" : "+s"(kmask), "+s"(k0), "+s"(k1));
        const int64_t g = g0 + step;
        if constexpr (RP) {
#pragma unroll
            for (int b = 0; b < B; ++b) replay_next[b] = replay_ahead[b];
            if (step + 1 < n_steps) replay_load(g + 1, replay_ahead);
        }
        const bool even = (g & 1) == 0;  // wave-uniform
        const int64_t kp = g >> 1;       // step pair: counter step word of the random streams

        // The counts that substep 3 takes from the post-hop state: a hop moves
        // a spring but never fills or frees a slot, so they are those of the
        // state before the step, and the thresholds' LDS reads are issued here.
        int z = 0;
        int first_empty = kCap;  // lowest empty slot of the chain (K = 1 rule)
#pragma unroll
        for (int b = 0; b < B && !RP; ++b) {
            z += __popcll(__ballot(s[b] >= 0) & seg_mask<W>(sb));
            if constexpr (K1) {
                const uint64_t m = __ballot(s[b] < 0 && li * B + b < n) & seg_mask<W>(sb);
                if (m) first_empty = min(first_empty, ((int)__builtin_ctzll(m) - sb) * B + b);
            }
        }
        const int K = K1 ? (z < n ? 1 : 0) : n - z;
        const uint32_t t1 = thr[K < 0 ? 0 : K];
        const uint32_t t2 = thr[kMaxBeads + 1 + (K < 0 ? 0 : K)];

        // ---- substep 1a: slip-spring force, sum of d_j over the springs of each
        // bead in increasing slot order.  Every occupied slot sets its bit in
        // its bead's slot mask (LDS atomics of one wavefront complete in
        // order, so the clearing stores land first); each bead then reads its
        // mask and adds the staged offsets of its set bits lowest first.  The
        // mask round trip is issued before the step's noise is computed (it
        // does not depend on it), so that its latency runs under that
        // arithmetic; the first two offsets of every bead are read together.
        SlotMask<kCap> mw[B];
#pragma unroll
        for (int b = 0; b < B; ++b)
#pragma unroll
            for (int w = 0; w < kMaskWords; ++w) lmask_store(&lmask[mask_at(li * B + b, w)], 0u);
#pragma unroll
        for (int b = 0; b < B; ++b)
            if (s[b] >= 0) lmask_or(&lmask[mask_at(s[b], mbit_word[b])], mbit[b]);
#pragma unroll
        for (int b = 0; b < B; ++b)
#pragma unroll
            for (int w = 0; w < kMaskWords; ++w) mw[b].w[w] = lmask_load(&lmask[mask_at(li * B + b, w)]);

        // ---- substep 1b, first part: sqrt(2 dt) w of this step.
        v3<T> noise[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int i = li * B + b;
            if (even) {
                const uint4 x = draw(kNoise, (uint32_t)i, gid, kp, k0, k1);
                box_muller(x.x, x.y, cnoise, noise[b].x, noise[b].y);
                box_muller(x.z, x.w, cnoise, noise[b].z, carry_n[b]);
            } else {
                noise[b].x = carry_n[b];
                box_muller(carry_w0[b], carry_w1[b], cnoise, noise[b].y, noise[b].z);
            }
        }

        // ---- substep 1a, completion: the first two springs of every bead
        // (read unconditionally: a missing one reads the zero entry), then
        // the rare beads with more.  The sum is never -0, so adding +0 for a
        // missing spring changes nothing.
        v3<T> acc[B];
        bool more = false;
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const v3<T> o0 = unpack3(offs[mw[b].lowest()]);
            mw[b].drop();
            const v3<T> o1 = unpack3(offs[mw[b].lowest()]);
            mw[b].drop();
            acc[b] = (zero3<T>() + o0) + o1;
            more |= mw[b].any();
        }
        if (wave_any(more)) {
            do {
                more = false;
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    if (mw[b].any()) {
                        acc[b] = acc[b] + unpack3(offs[mw[b].lowest()]);
                        mw[b].drop();
                    }
                    more |= mw[b].any();
                }
            } while (wave_any(more));
        }

        // ---- substep 1b: Euler-Maruyama for beads, advection for anchors.
        // FP32 under flow: positions drift and stretch far from the origin
        // while bonds near the chain ends and anchor offsets stay O(1), so the
        // terms of the move that scale with |R| must keep their low bits:
        //  - beads: the flow term takes dt kappa (hi + lo); the low part's
        //    product is small but systematic and would add up over the steps;
        //  - anchors: advected error-free (flow_row, cadd_big); under shear an
        //    anchor's increment dt gamma_dot A_y is the same number every
        //    step, so its rounding error would add up linearly;
        //  - chains under elongation (a positive diagonal entry of kappa),
        //    which stretch to bonds of hundreds: the bead's flow term and its
        //    bond force, taken from the compensated positions, split into a
        //    binary32 value and its exact rounding error (flow_row,
        //    two_prod); the large part enters hi through an exact TwoSum
        //    (cadd_big), so that only O(1) quantities are ever rounded.
        // Which form a chain takes depends only on its own element, and chains
        // without flow keep the plain binary32 step, so trajectories do not
        // depend on the mapping or the launch split.
        auto plain_inc = [&](int b) {
            v3<T> inc = noise[b];
            inc = fma3(cbond, br[b] - bl[b], inc);
            return fma3(-cspring, acc[b], inc);
        };
        if constexpr (kComp) {
            if (flow) {  // wave-uniform
                if (wave_any(chain_stretch)) {
                    const v3<T> nh = from_next3(rh[0]), nl = from_next3(rl[0]);
                    const v3<T> ph = from_prev3(rh[B - 1]), pl = from_prev3(rl[B - 1]);
                    v3<T> lap[B];  // every bead reads its in-lane neighbours before any moves
#pragma unroll
                    for (int b = 0; b < B; ++b) {
                        const int i = li * B + b;
                        const v3<T> h1 = (b + 1 < B) ? rh[b + 1 < B ? b + 1 : b] : nh;
                        const v3<T> l1 = (b + 1 < B) ? rl[b + 1 < B ? b + 1 : b] : nl;
                        const v3<T> h0 = (b > 0) ? rh[b > 0 ? b - 1 : 0] : ph;
                        const v3<T> l0 = (b > 0) ? rl[b > 0 ? b - 1 : 0] : pl;
                        const bool right = i < n - 1, left = i > 0;
                        // (R_{i+1} - R_i) - (R_i - R_{i-1}) from the compensated parts
                        lap[b] = (sel(right, h1 - rh[b], zero3<T>()) - sel(left, rh[b] - h0, zero3<T>())) +
                                 (sel(right, l1 - rl[b], zero3<T>()) - sel(left, rl[b] - l0, zero3<T>()));
                    }
#pragma unroll
                    for (int b = 0; b < B; ++b) {
                        if (li * B + b < n && chain_stretch) {
                            const v3<T> rest = fma3(-cspring, acc[b], noise[b]);
                            v3<T> big, small;
                            flow_row<0>(kdt, kmask, rh[b], rl[b], big.x, small.x);
                            flow_row<1>(kdt, kmask, rh[b], rl[b], big.y, small.y);
                            flow_row<2>(kdt, kmask, rh[b], rl[b], big.z, small.z);
                            cadd_force(rh[b].x, rl[b].x, big.x, small.x, cbond, lap[b].x, rest.x);
                            cadd_force(rh[b].y, rl[b].y, big.y, small.y, cbond, lap[b].y, rest.y);
                            cadd_force(rh[b].z, rl[b].z, big.z, small.z, cbond, lap[b].z, rest.z);
                        }
                    }
                }
                // The tests of kmask (wave-uniform) stay outside the
                // per-lane conditions: nested inside them they would be
                // turned into lane masks and vector selects.
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const v3<T> f = masked_mat3(kdt, kmask, rh[b], rl[b]);
                    if (li * B + b < n && !chain_stretch) {
                        v3<T> inc = plain_inc(b);
                        if (chain_flow) inc = inc + f;
                        cadd3(rh[b], rl[b], inc);
                    }
                }
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const bool adv = s[b] >= 0 && chain_flow;
                    v3<T> big, small;
                    if (any_bits(kmask, 0x007u)) {
                        flow_row<0>(kdt, kmask, ah[b], al[b], big.x, small.x);
                        if (adv) cadd_big(ah[b].x, al[b].x, big.x, small.x);
                    }
                    if (any_bits(kmask, 0x038u)) {
                        flow_row<1>(kdt, kmask, ah[b], al[b], big.y, small.y);
                        if (adv) cadd_big(ah[b].y, al[b].y, big.y, small.y);
                    }
                    if (any_bits(kmask, 0x1C0u)) {
                        flow_row<2>(kdt, kmask, ah[b], al[b], big.z, small.z);
                        if (adv) cadd_big(ah[b].z, al[b].z, big.z, small.z);
                    }
                }
            } else {
#pragma unroll
                for (int b = 0; b < B; ++b)
                    if (li * B + b < n) cadd3(rh[b], rl[b], plain_inc(b));
            }
        } else {
#pragma unroll
            for (int b = 0; b < B; ++b) {
                v3<T> inc = plain_inc(b);
                // wave-uniform branch; fma(0, r, x) = x keeps chains without flow bit-identical
                if (flow) inc = fma_mat3(kdt, rh[b], inc);
                if (li * B + b < n) rh[b] = rh[b] + inc;
            }
            if (flow) {
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const v3<T> A = ah[b];
                    const v3<T> inc = {kdt[0] * A.x + kdt[1] * A.y + kdt[2] * A.z,
                                       kdt[3] * A.x + kdt[4] * A.y + kdt[5] * A.z,
                                       kdt[6] * A.x + kdt[7] * A.y + kdt[8] * A.z};
                    if (s[b] >= 0) ah[b] = ah[b] + inc;
                }
            }
        }
        bonds_and_records();

        // ---- substep 2: hops from the post-move positions.
        uint32_t wrec[B];  // reconstruction words
        int s_rec[B];      // replay: the recorded slot state after this step
        if constexpr (RP) {
            bool bad = false;
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const int j = li * B + b;
                s_rec[b] = -1;
                wrec[b] = 0u;
                if (even) {  // the pair's carried normals still come from NOISE2
                    const uint4 y = draw(kNoise2, (uint32_t)j, gid, kp, k0, k1);
                    carry_w0[b] = y.x;
                    carry_w1[b] = y.y;
                }
                if (j < n) {
                    const int v = replay_next[b];
                    // a creation lands on an end; a destruction leaves an end after the hop, so
                    // a bead within one of it; anything else moves by at most one bead
                    const bool ok = s[b] >= 0 ? (v == -1 ? (s[b] <= 1 || s[b] >= n - 2)
                                                         : (v >= s[b] - 1 && v <= s[b] + 1 && v < n))
                                              : (v == -1 || v == 0 || v == n - 1);
                    bad |= !ok;
                    s_rec[b] = ok ? v : s[b];
                }
            }
            if (bad) atomicOr(a.flags, kFlagReplay);
        }
#pragma unroll
        for (int b = 0; b < B && !RP; ++b) {
            const int j = li * B + b;
            uint32_t whop;
            if (even) {
                const uint4 y = draw(kNoise2, (uint32_t)j, gid, kp, k0, k1);
                whop = y.z;
                wrec[b] = y.w;
                carry_w0[b] = y.x;
                carry_w1[b] = y.y;
            } else {
                const uint4 z = draw(kSlot, (uint32_t)j, gid, kp, k0, k1);
                whop = z.x;
                wrec[b] = z.y;
            }
            const int t = s[b] > 0 ? s[b] : 0;
            const BeadRec<T> r = rec[lbase + t];
            const v3<T> Rh = {r.v[0], r.v[1], r.v[2]};
            const v3<T> Rl = {r.v[3], r.v[4], r.v[5]};
            const v3<T> bp = {r.v[6], r.v[7], r.v[8]};      // R_{S+1} - R_S
            const v3<T> bm = {-r.v[9], -r.v[10], -r.v[11]};  // R_{S-1} - R_S
            const v3<T> dd = (Rh - ah[b]) + (Rl - al[b]);
            // (R_{S+-1} - A)^2 - (R_S - A)^2 = b (b + 2 d) with b = R_{S+-1} - R_S
            const T up = dot(bp, bp + T(2) * dd);
            const T dn = dot(bm, bm + T(2) * dd);
            const T pp = (t < n - 1) ? glauber(up, hop_e2q, hop_h2) : T(0);
            const T pm = (t > 0) ? glauber(dn, hop_e2q, hop_h2) : T(0);
            const T u = u01<T>(whop);
            if (s[b] >= 0) {
                if (u < pp)
                    s[b] = t + 1;
                else if (u < pp + pm)
                    s[b] = t - 1;
            }
        }

        // ---- substep 3: destruction at the ends and construction, all from the
        // post-hop state.  K = C - Z attempts (every empty slot once), or with
        // the K = 1 rule a single attempt by the segment's lowest empty slot
        // (both counted at the start of the step).
        int create_at[B];
        bool destroyed[B];
        bool any_create = false;
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int j = li * B + b;
            const uint32_t uw = wrec[b] >> 9;
            create_at[b] = -1;
            destroyed[b] = false;
            if constexpr (RP) {
                if (s[b] < 0) {
                    create_at[b] = s_rec[b];
                } else {
                    destroyed[b] = s_rec[b] < 0;
                    s[b] = s_rec[b];
                }
            } else if (j < n) {
                if (s[b] >= 0) {
                    if ((s[b] == 0 || s[b] == n - 1) && uw < a.thr_destroy) {
                        s[b] = -1;
                        destroyed[b] = true;
                    }
                } else if (!K1 || j == first_empty) {
                    if (uw < t1)
                        create_at[b] = 0;
                    else if (uw < t2)
                        create_at[b] = n - 1;
                }
            }
            any_create |= create_at[b] >= 0;
        }
        if (wave_any(any_create)) {
#pragma unroll
            for (int b = 0; b < B; ++b) {
                const int j = li * B + b;
                if (create_at[b] >= 0) {
                    const BeadRec<T> r = rec[lbase + create_at[b]];
                    const v3<T> Rh = {r.v[0], r.v[1], r.v[2]};
                    const v3<T> Rl = {r.v[3], r.v[4], r.v[5]};
                    const v3<T> off3 = asd * normals3<T>(draw(kAnchor, (uint32_t)j, gid, g, k0, k1));
                    if constexpr (kComp) {
                        ah[b] = Rh;
                        al[b] = Rl;
                        cadd3(ah[b], al[b], off3);
                    } else {
                        ah[b] = Rh + off3;
                    }
                    s[b] = create_at[b];
                }
            }
        }
        refresh_offsets();

        if (a.rec_s) {
            int8_t* row = a.rec_s + (g + 1 - a.rec_g0) * a.total + off;
#pragma unroll
            for (int b = 0; b < B; ++b)
                if (li * B + b < n) row[li * B + b] = (int8_t)s[b];
        }
        if constexpr (kTraj) {
            store_r(step + 1);
            if constexpr (RP) {
#pragma unroll
                for (int b = 0; b < B; ++b)
                    if (destroyed[b]) store_a(step + 1, b);
            } else {
                log_destroyed(destroyed);
            }
        }

        // ---- observables of the new state.
        if (!RP && a.sample_every > 0 && phase == 0) {  // a replay samples nothing
            const double kss = 3.0 / a.ph.ns;
            // Lane partials go to LDS in two groups of six as they are formed,
            // so that the twelve FP64 sums are never live together (otherwise
            // the sampling step sets the kernel's register peak).  Then a
            // transpose: lane li of a segment sums values li, li + W, ... over
            // the segment's lanes in lane order (deterministic).
            double* mine = sums + lane * kSampleValues;
            {
                double p[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const double bx = br[b].x, by = br[b].y, bz = br[b].z;  // zero past the end
                    p[0] += 3.0 * bx * bx;
                    p[1] += 3.0 * by * by;
                    p[2] += 3.0 * bz * bz;
                    p[3] += 3.0 * bx * by;
                    p[4] += 3.0 * by * bz;
                    p[5] += 3.0 * bz * bx;
                }
#pragma unroll
                for (int q = 0; q < 6; ++q) mine[q] = p[q];
            }
            {
                double p[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const double dx = d[b].x, dy = d[b].y, dz = d[b].z;  // zero when empty
                    p[0] += kss * dx * dx;
                    p[1] += kss * dy * dy;
                    p[2] += kss * dz * dz;
                    p[3] += kss * dx * dy;
                    p[4] += kss * dy * dz;
                    p[5] += kss * dz * dx;
                }
#pragma unroll
                for (int q = 0; q < 6; ++q) mine[6 + q] = p[q];
            }
            int z2 = 0;
#pragma unroll
            for (int b = 0; b < B; ++b) z2 += __popcll(__ballot(s[b] >= 0) & seg_mask<W>(sb));
            wave_sync();
#pragma unroll
            for (int v = li; v < kSampleValues; v += W) {
                double tot = 0.0;
#pragma unroll 8
                for (int r = 0; r < W; ++r) tot += sums[(sb + r) * kSampleValues + v];
                const double corr = (v < 3) ? (double)n : (v >= 6 && v < 9) ? (double)z2 : 0.0;
                if (valid) a.samples[(q_launch * a.n_chains + chain) * kSampleValues + v] = tot - corr;
            }
            ++q_launch;
            wave_sync();  // the records are rewritten by the next step
        }
        if (a.sample_every > 0) phase = (phase + 1 == a.sample_every) ? 0 : phase + 1;
    }

    // The final state goes back to the state buffer, except from a replay,
    // which reads its checkpoint in place and leaves it for later reverse
    // passes (its output is the trajectory).
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int i = li * B + b;
        if (i < n) {
            finite_ok &= finite3(rh[b]);
            if constexpr (!RP) {
                st3<T>(a.st.r0, off + i, rh[b]);
                st3<T>(a.st.a0, off + i, ah[b]);
                if constexpr (kComp) {
                    st3<T>(a.st.r1, off + i, rl[b]);
                    st3<T>(a.st.a1, off + i, al[b]);
                }
                a.st.s[off + i] = s[b];
            }
        }
    }
    // a second copy of the final state when asked (the next checkpoint of a
    // recorded window)
    if (!RP && a.ck_end.r0) {
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int i = li * B + b;
            if (i < n) {
                st3<T>(a.ck_end.r0, off + i, rh[b]);
                st3<T>(a.ck_end.a0, off + i, ah[b]);
                if constexpr (kComp) {
                    st3<T>(a.ck_end.r1, off + i, rl[b]);
                    st3<T>(a.ck_end.a1, off + i, al[b]);
                }
                a.ck_end.s[off + i] = s[b];
            }
        }
    }
    if constexpr (RP) {
#pragma unroll
        for (int b = 0; b < B; ++b)
            if (li * B + b < n) store_a(n_steps, b);
    }
    if constexpr (ST) {
#pragma unroll
        for (int b = 0; b < B; ++b)
            if (li * B + b < n) reinterpret_cast<v3<T>*>(a.traj2)[off + li * B + b] = ah[b] + al[b];
        if (valid && li == 0) a.dcnt[chain] = dcount;
    }
    if (!finite_ok) atomicOr(a.flags, kFlagNonFinite);
    };  // run

    if constexpr (PS) {
        static_assert(!RP && !ST, "the persistent schedule runs plain steps only");
        {
            // Persistent schedule (a plain step launch): the units (time chunk
            // c, wave task w) are taken in the order c * n_wt + w from one
            // counter, and a unit waits until unit (c - 1, w) has stored its
            // chains' state.  Every unit's predecessor was taken earlier, by a
            // wavefront that is running, and the earliest unfinished unit
            // never waits, so the queue drains; all wavefronts stay busy to
            // the end instead of the last round of a one-wave-per-task launch
            // running part-full.
            const int64_t g0 = a.ctrl[kCtrlSteps];
            const int64_t n_wt = a.n_wave_tasks;
            const int32_t L = a.chunk;
            const int64_t n_chunks = (a.n_steps + L - 1) / L;
            const int64_t total = n_wt * n_chunks;
            uint32_t* progress = a.sched + 1;  // [n_wt] chunks finished per wave task
            for (;;) {
                uint32_t u = 0;
                if (lane == 0) u = atomicAdd(a.sched, 1u);
                u = __builtin_amdgcn_readfirstlane(u);
                if ((int64_t)u >= total) break;
                const int64_t c = (int64_t)u / n_wt, w = (int64_t)u % n_wt;
                if (c > 0) {
                    // bounded wait (the bound only guards against a hang: the
                    // predecessor is running and finishes within one unit)
                    for (uint32_t spin = 0;; ++spin) {
                        const uint32_t done = __hip_atomic_load(&progress[w], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
                        if (__builtin_amdgcn_readfirstlane(done) >= (uint32_t)c) break;
                        if (spin > (1u << 22)) {
                            if (lane == 0) atomicOr(a.flags, kFlagInternal);
                            break;
                        }
                        __builtin_amdgcn_s_sleep(8);
                    }
                }
                const int64_t gs = g0 + c * L;
                const int32_t ns = (int32_t)min((int64_t)L, (int64_t)a.n_steps - c * L);
                // samples of steps g0 .. gs - 1 precede this unit's: steps g with (g + 1) % n_s == 0
                const int64_t q0 = a.sample_every > 0 ? gs / a.sample_every - g0 / a.sample_every : 0;
                run(w, gs, ns, q0);
                __hip_atomic_store(&progress[w], (uint32_t)(c + 1), __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    } else {
        run((int64_t)blockIdx.x * kWavesPerGroup + wv, a.ctrl[kCtrlSteps], a.n_steps, 0);
    }
}

// Waves per SIMD the register budget must allow.  The step is held one wave
// above what its registers would give: FP32 with one bead per lane at 5 waves
// (96 VGPRs instead of 106), with two at 4 (128 instead of 138), FP64 with
// one at 3 (168 instead of ~225).  The compiler spills a few values, mostly
// reloaded in the sampling step and the launch epilogue; the extra wave hides
// more of the LDS round trips (16384 x 32 FP32: 18.1 -> 17.5 ms per 5000-step
// launch; 16384 x 128 at 64 x 2: 31.9 -> 27.0 ms per 2000 steps; 16384 x 32
// FP64: 13.9 -> 12.7 ms per 1000 steps).  Two-bead FP64 cannot reach 3
// waves and is left to the compiler.
template <typename T, int B>
constexpr int kStepWavesPerEu = std::is_same<T, float>::value ? (B == 1 ? 5 : 4) : (B == 1 ? 3 : 1);

template <typename T, int W, int B, bool K1, bool ST, bool FL>
__global__ void __launch_bounds__(kGroupThreads) __attribute__((amdgpu_waves_per_eu(kStepWavesPerEu<T, B>)))
k_step(StepArgs a)
{
    step_body<T, W, B, K1, false, ST, FL, false>(a);
}

// The same step under the persistent schedule (plain steps: nothing recorded
// or stored), a kernel of its own so that the queue's registers do not weigh
// on the other variants.
template <typename T, int W, int B, bool K1, bool FL>
__global__ void __launch_bounds__(kGroupThreads) __attribute__((amdgpu_waves_per_eu(kStepWavesPerEu<T, B>)))
k_step_queue(StepArgs a)
{
    step_body<T, W, B, K1, false, false, FL, true>(a);
}

// Replay of recorded slot rows (the adjoint's reverse pass re-creates each
// segment's trajectory this way).  It samples no stress.  FP32 with one bead
// per lane is held at 5 waves per SIMD (84 VGPRs, no spills): at 6 it spills
// a few values, and every reload from scratch waits for all of the wave's
// memory operations in flight, the trajectory stores included.
template <typename T, int W, int B, bool FL>
__global__ void __launch_bounds__(kGroupThreads) __attribute__((amdgpu_waves_per_eu(std::is_same<T, float>::value && B == 1 ? 5 : 1)))
k_replay(StepArgs a)
{
    step_body<T, W, B, false, true, false, FL, false>(a);
}

// Workgroups of the queue kernel that fit on the device at once (occupancy x
// CUs), looked up once per kernel.
template <typename T, int W, int B, bool K1, bool FL> int resident_groups()
{
    static int cached = 0;
    if (cached == 0) {
        int per_cu = 0, dev = 0, cus = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_step_queue<T, W, B, K1, FL>, kGroupThreads, 0) !=
                hipSuccess ||
            hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
            return 0;
        cached = per_cu * cus;
    }
    return cached;
}

// Shortest time chunk of the persistent schedule, in steps.
constexpr int kMinChunkSteps = 200;

template <typename T, int W, int B, bool FL> hipError_t launch_f(const StepArgs& a, dim3 grid, hipStream_t s)
{
    if (a.sched && !a.replay_s && !a.traj) {
        // persistent: as many groups as fit, each wave taking units from the queue
        auto kern = a.construct_rule == 1 ? k_step_queue<T, W, B, true, FL> : k_step_queue<T, W, B, false, FL>;
        const int r = a.construct_rule == 1 ? resident_groups<T, W, B, true, FL>() : resident_groups<T, W, B, false, FL>();
        StepArgs p = a;
        // time chunks per wave task: the count (1..16, chunks of at least
        // kMinChunkSteps) with the shortest estimated run, in units of the
        // launch's length.  The slots take ceil(units / slots) rounds of units
        // of 1/nc of the steps, but a wave task's chunks run one after
        // another, so never fewer than nc rounds; each chunk is also charged a
        // little for re-reading and writing the state.  With fewer wave tasks
        // than slots this keeps one chunk: more would only park wavefronts
        // that wait for their chains' previous chunk.
        const double slots = (double)std::max(1, r) * kWavesPerGroup;
        int best = 1;
        double best_t = 1e30;
        for (int nc = 1; nc <= 16; ++nc) {
            if (nc > 1 && (a.n_steps + nc - 1) / nc < kMinChunkSteps) break;
            const double rounds = std::max(std::ceil((double)(a.n_wave_tasks * nc) / slots), (double)nc);
            const double t = rounds / nc + 0.002 * nc;
            if (t < best_t - 1e-12) {
                best_t = t;
                best = nc;
            }
        }
        p.chunk = (a.n_steps + best - 1) / best;
        if (p.chunk < 1) p.chunk = 1;
        const int64_t units = a.n_wave_tasks * ((a.n_steps + p.chunk - 1) / p.chunk);
        const int64_t need = (units + kWavesPerGroup - 1) / kWavesPerGroup;
        const dim3 pg((unsigned)std::max<int64_t>(1, std::min<int64_t>(r > 0 ? r : need, need)));
        hipLaunchKernelGGL(kern, pg, dim3(kGroupThreads), 0, s, p);
        return hipGetLastError();
    }
    if (a.replay_s)
        hipLaunchKernelGGL((k_replay<T, W, B, FL>), grid, dim3(kGroupThreads), 0, s, a);
    else if (a.traj && a.construct_rule == 1)
        hipLaunchKernelGGL((k_step<T, W, B, true, true, FL>), grid, dim3(kGroupThreads), 0, s, a);
    else if (a.traj)
        hipLaunchKernelGGL((k_step<T, W, B, false, true, FL>), grid, dim3(kGroupThreads), 0, s, a);
    else if (a.construct_rule == 1)
        hipLaunchKernelGGL((k_step<T, W, B, true, false, FL>), grid, dim3(kGroupThreads), 0, s, a);
    else
        hipLaunchKernelGGL((k_step<T, W, B, false, false, FL>), grid, dim3(kGroupThreads), 0, s, a);
    return hipGetLastError();
}

// A null velocity-gradient table means a run at rest: the variant without the
// flow terms.
template <typename T, int W, int B> hipError_t launch_t(const StepArgs& a, hipStream_t s)
{
    constexpr int kChainsPerGroup = kWavesPerGroup * (kWaveSize / W);
    const int64_t groups = (a.n_tasks + kChainsPerGroup - 1) / kChainsPerGroup;
    if (groups == 0) return hipSuccess;
    const dim3 grid((unsigned)groups);
    return a.kappa ? launch_f<T, W, B, true>(a, grid, s) : launch_f<T, W, B, false>(a, grid, s);
}

template <typename T> hipError_t launch_p(int W, int B, const StepArgs& a, hipStream_t s)
{
    if (B == 1) {
        switch (W) {
        case 8: return launch_t<T, 8, 1>(a, s);
        case 16: return launch_t<T, 16, 1>(a, s);
        case 32: return launch_t<T, 32, 1>(a, s);
        case 64: return launch_t<T, 64, 1>(a, s);
        }
    } else if (B == 2) {
        switch (W) {
        case 16: return launch_t<T, 16, 2>(a, s);
        case 32: return launch_t<T, 32, 2>(a, s);
        case 64: return launch_t<T, 64, 2>(a, s);
        }
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_step(int precision, int W, int B, const StepArgs& a, hipStream_t s)
{
    return precision == 0 ? launch_p<float>(W, B, a, s) : launch_p<double>(W, B, a, s);
}

}  // namespace ssp
