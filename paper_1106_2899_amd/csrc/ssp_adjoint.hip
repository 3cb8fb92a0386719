// Discrete adjoint of the Euler map of Sec. 3.1 over a recorded window,
// conditioned on the recorded slot trajectory (hops, creations,
// destructions) and on the random normals: the pathwise derivative of a
// final stress component J = sigma_c(R_T) of every chain with respect to the
// velocity gradient kappa (all nine entries) and the slip-spring strength
// N_s.  One launch processes one checkpoint segment backwards, reading the
// positions that the replay of the segment stored (k_replay) and rebuilding
// the anchors from the few the replay stored.
//
// Per step m of the segment (state before the step: R_m, A_m, slots S_m;
// after: S_{m+1}), with lR = dJ/dR_{m+1}, lA = dJ/dA_{m+1}:
//   created slots (S_m < 0 <= S_{m+1}):  lR[S_{m+1}] += lA,
//                                         dJ/dN_s += lA . g / (2 sqrt(3 N_s));
//   dJ/dN_s    += dt (3/N_s^2) lR[S_m] . (R_m[S_m] - A_m)        (occupied),
//   dJ/dkappa  += dt (lR (x) R_m + lA (x) A_m)                    (surviving slots),
//   dJ/dA_m     = (1 + dt kappa^T) lA (surviving) + dt (3/N_s) lR[S_m],
//   dJ/dR_m     = lR + dt (L lR - (3/N_s) c lR + kappa^T lR),
// L the free-end bond Laplacian (stiffness 3) and c the springs per bead.
#include <mutex>
#include <type_traits>
#include <vector>

#include "ssp_device.h"
#include "ssp_internal.h"

namespace ssp {

namespace {

template <typename T> struct alignas(16) AdjRec {
    T v[8];  // lR (3), R_m (3), padding
};

__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ float lane_value(float v, int l)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ __forceinline__ double lane_value(double v, int l)
{
    const int2 p = __builtin_bit_cast(int2, v);
    return __builtin_bit_cast(double, make_int2(__builtin_amdgcn_readlane(p.x, l), __builtin_amdgcn_readlane(p.y, l)));
}

template <typename T> __device__ __forceinline__ v3<T> kT(const T (&k)[9], v3<T> l)
{
    return {k[0] * l.x + k[3] * l.y + k[6] * l.z, k[1] * l.x + k[4] * l.y + k[7] * l.z,
            k[2] * l.x + k[5] * l.y + k[8] * l.z};
}

template <typename T> __device__ __forceinline__ T comp_of(v3<T> v, int c)
{
    return c == 0 ? v.x : (c == 1 ? v.y : v.z);
}

// d sigma_ab / d b for sigma_ab = 3 b_a b_b.
template <typename T> __device__ __forceinline__ v3<T> dsigma(v3<T> b, int ca, int cb)
{
    v3<T> g = zero3<T>();
    const T va = T(3) * comp_of(b, cb), vb = T(3) * comp_of(b, ca);
    if (ca == 0) g.x += va;
    if (ca == 1) g.y += va;
    if (ca == 2) g.z += va;
    if (cb == 0) g.x += vb;
    if (cb == 1) g.y += vb;
    if (cb == 2) g.z += vb;
    return g;
}

// SW: a stored window (one segment written by the storing forward): the
// end-of-window anchors come from a single plane and destroyed springs'
// anchors from the per-chain log, read back from its end; every pair of
// consecutive slot rows is checked to be a move the step can make.  Without
// SW (a replayed segment) only the segment's first step is checked: the replay
// checks the rest of the segment it re-creates, from its checkpoint.
template <typename T, int W, int B, bool SW>
__global__ void __launch_bounds__(kGroupThreads) k_adjoint(AdjointArgs a)
{
    constexpr int kChainsPerWave = kWaveSize / W;
    constexpr int kCap = W * B;
    __shared__ AdjRec<T> lds_rec[kWavesPerGroup][kWaveSize * B];
    __shared__ uint32_t lds_cnt[kWavesPerGroup][kWaveSize * B];
    __shared__ double lds_sum[kWavesPerGroup][kWaveSize * 10];

    const int lane = threadIdx.x & (kWaveSize - 1);
    const int wv = threadIdx.x / kWaveSize;
    const int li = lane % W;
    const int seg = lane / W;
    const int sb = lane - li;
    const int64_t task = ((int64_t)blockIdx.x * kWavesPerGroup + wv) * kChainsPerWave + seg;
    const bool valid = task < a.n_tasks;
    int chain = valid ? a.tasks[task] : 0;
    int n = valid ? a.ct.n[chain] : 0;
    int64_t off = valid ? a.ct.off[chain] : 0;
    uint32_t gid = valid ? a.ct.gid[chain] : 0u;
    int elem = valid ? a.ct.elem[chain] : 0;
    if constexpr (W == kWaveSize) {
        // one chain per wavefront: its table entries go to scalar registers
        chain = wave_uniform(chain);
        n = wave_uniform(n);
        off = wave_uniform(off);
        gid = wave_uniform(gid);
        elem = wave_uniform(elem);
    }
    const int lbase = seg * kCap;
    AdjRec<T>* rec = lds_rec[wv];
    uint32_t* cnt = lds_cnt[wv];
    double* sums = lds_sum[wv];

    const T dt = T(a.ph.dt);
    const T ks = T(3.0 / a.ph.ns);
    const double dsig = 1.0 / (2.0 * sqrt(3.0 * a.ph.ns));
    const double kns = a.ph.dt * 3.0 / (a.ph.ns * a.ph.ns);
    const double ddt = a.ph.dt;
    T kap[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        kap[q] = (valid && a.kappa) ? T(a.kappa[9 * elem + q]) : T(0);  // no table: at rest
        // one chain per wavefront: its element's kappa is wave-uniform
        if constexpr (W == kWaveSize) kap[q] = wave_uniform(kap[q]);
    }
    const v3<T>* trajR = reinterpret_cast<const v3<T>*>(a.traj);
    const v3<T>* trajA = reinterpret_cast<const v3<T>*>(a.traj2);
    T* lam = reinterpret_cast<T*>(a.lam);

    // Anchors run backwards: a spring that survives step m was only advected,
    // A_{m+1} = (I + K) A_m with K = dt kappa as the step kernel rounds it, so
    // A_m = A_{m+1} + D A_{m+1}, D = (I + K)^{-1} - I = -(I + K)^{-1} K.  D is
    // O(dt kappa), so D A in T costs no precision; A itself is carried in
    // FP64.  Anchors of destroyed springs and those at the segment end are
    // read from the replay output.
    T dinv[9];
    {
        double K[9], M[9], Mi[9];
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            K[q] = (valid && a.kappa) ? (double)T(a.ph.dt * a.kappa[9 * elem + q]) : 0.0;
            M[q] = K[q] + ((q % 4 == 0) ? 1.0 : 0.0);
        }
        Mi[0] = M[4] * M[8] - M[5] * M[7];
        Mi[1] = M[2] * M[7] - M[1] * M[8];
        Mi[2] = M[1] * M[5] - M[2] * M[4];
        Mi[3] = M[5] * M[6] - M[3] * M[8];
        Mi[4] = M[0] * M[8] - M[2] * M[6];
        Mi[5] = M[2] * M[3] - M[0] * M[5];
        Mi[6] = M[3] * M[7] - M[4] * M[6];
        Mi[7] = M[1] * M[6] - M[0] * M[7];
        Mi[8] = M[0] * M[4] - M[1] * M[3];
        const double det = M[0] * Mi[0] + M[1] * Mi[3] + M[2] * Mi[6];
#pragma unroll
        for (int r = 0; r < 3; ++r)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                dinv[3 * r + c] = T(-(Mi[3 * r] * K[c] + Mi[3 * r + 1] * K[3 + c] + Mi[3 * r + 2] * K[6 + c]) / det);
        if constexpr (W == kWaveSize) {
#pragma unroll
            for (int q = 0; q < 9; ++q) dinv[q] = wave_uniform(dinv[q]);
        }
    }
    const int ca = (a.comp < 3) ? a.comp : (a.comp == 3 ? 0 : (a.comp == 4 ? 1 : 2));
    const int cb = (a.comp < 3) ? a.comp : (a.comp == 3 ? 1 : (a.comp == 4 ? 2 : 0));

    auto traj_r = [&](int row, int i) -> v3<T> { return trajR[(int64_t)row * a.total + off + i]; };

    v3<T> lR[B], lA[B];
    if (a.seed_lambda) {
        v3<T> R[B], br[B], bl[B];
#pragma unroll
        for (int b = 0; b < B; ++b) R[b] = (li * B + b < n) ? traj_r(a.len, li * B + b) : zero3<T>();
        const v3<T> nx = from_next3(R[0]);
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int i = li * B + b;
            const v3<T> h = (b + 1 < B) ? R[b + 1 < B ? b + 1 : b] : nx;
            br[b] = (i < n - 1) ? (h - R[b]) : zero3<T>();
        }
        const v3<T> left = from_prev3(br[B - 1]);
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int i = li * B + b;
            bl[b] = (i > 0 && i < n) ? ((b > 0) ? br[b > 0 ? b - 1 : 0] : left) : zero3<T>();
            lR[b] = (i < n) ? (dsigma(bl[b], ca, cb) - dsigma(br[b], ca, cb)) : zero3<T>();
            lA[b] = zero3<T>();
        }
    } else {
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int i = li * B + b;
            if (i < n) {
                const T* p = lam + (off + i) * 6;
                lR[b] = {p[0], p[1], p[2]};
                lA[b] = {p[3], p[4], p[5]};
            } else {
                lR[b] = zero3<T>();
                lA[b] = zero3<T>();
            }
        }
    }

    double G[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) G[q] = 0.0;
    double Gns = 0.0;
    // The per-step gradient terms dt (lR (x) R_m + lA (x) A_m) and
    // dt (3/N_s^2) lR[S_m] . (R_m[S_m] - A_m) are summed in the path's
    // precision over blocks of kBlock steps (without the constant factors),
    // and each block's sums are added to the FP64 totals: a block's sum holds
    // at most 2 kBlock rounding errors of its own size, and the conversions
    // and FP64 arithmetic run once per block instead of once per step.
    constexpr int kBlock = 16;
    T Gp[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) Gp[q] = T(0);
    T Gnsp = T(0);
    int in_block = 0;

    // Step m reads the slot rows m and m + 1 and the trajectory row m.  Row
    // m + 1 of the slots is row m of the step after, carried; row m and the
    // trajectory are loaded kAhead steps ahead, so that their latency runs
    // under the arithmetic of the steps before.
    // Recorded slot rows are checked before use as LDS indices (where they are
    // used, not where they are loaded, so that a prefetch is not waited for):
    // a value outside -1..n-1 reads as an empty slot and latches kFlagReplay.
    // So does a pair of rows no step can produce (a spring that moves by more
    // than one bead, is created away from an end, or is destroyed more than
    // one bead away from an end, where no hop can take it): checked at every step
    // with SW, otherwise at the segment's first.  With SW, so does a log that
    // holds other than exactly one entry per destruction the rows show.
    bool bad_row = false;
    auto checked = [&](int v) -> int {
        const bool ok = v >= -1 && v < n;
        bad_row |= !ok;
        return ok ? v : -1;
    };
    auto row_at = [&](int64_t r, int i) -> int { return checked(a.rec_s[r * a.total + off + i]); };
    // rows in flight: ring slot q holds the rows len - 1 - q - kAhead k
    constexpr int kAhead = 3;
    int s_next[B], s_pre[kAhead][B];
    v3<T> R_pre[kAhead][B];
    // The loads are unconditional (a row before the window reads row 0, a
    // lane past the chain's end its first bead) and lanes past the end are
    // masked where the values are used: a load whose result is merged with
    // a default would be waited for at once.
    auto prefetch = [&](int q, int m) {
        const int row = m > 0 ? m : 0;
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int i = li * B + b < n ? li * B + b : 0;
            s_pre[q][b] = a.rec_s[(a.m0 + row) * a.total + off + i];  // checked when used
            R_pre[q][b] = traj_r(row, i);
        }
    };
    v3<double> Ac[B];  // A_{m+1} of the springs alive after step m
#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int i = li * B + b;
        s_next[b] = (i < n) ? row_at(a.m0 + a.len, i) : -1;
        Ac[b] = {0.0, 0.0, 0.0};
        if (i < n) {
            const v3<T> v = SW ? trajA[off + i] : trajA[(int64_t)a.len * a.total + off + i];
            Ac[b] = {(double)v.x, (double)v.y, (double)v.z};
        }
    }
    int64_t dcount = 0;  // SW: destruction-log entries not yet consumed
    if constexpr (SW) {
        dcount = valid ? a.dcnt[chain] : 0;
        if (dcount > a.dcap) atomicOr(a.flags, kFlagLogOverflow);
    }
    const v3<T>* dlog = SW ? reinterpret_cast<const v3<T>*>(a.dlog) + (int64_t)chain * a.dcap : nullptr;
    const uint64_t segm = W == kWaveSize ? ~0ull : (((1ull << W) - 1ull) << sb);
#pragma unroll
    for (int q = 0; q < kAhead; ++q) prefetch(q, a.len - 1 - q);

    // One step of the reverse recursion; row m sits in ring slot QC::value.
    // The loop below is unrolled over the ring, so that no register of a load
    // still in flight is copied (a copy would wait for the load).
    auto step_back = [&](const int m, auto QC) {
        constexpr int qs = decltype(QC)::value;
        const int64_t mg = a.m0 + m;
        // The ring's last slot is refilled at the start of the step, into
        // fresh registers: at the loop's wrap-around the compiler moves that
        // slot's registers, which waits for its load, and the load has then
        // had a whole step to arrive.  The other slots are refilled at the
        // end of their step, in place.
        int s_cur[B];
        v3<T> R_cur[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            s_cur[b] = s_pre[qs][b];
            R_cur[b] = R_pre[qs][b];
        }
        if constexpr (qs == kAhead - 1) prefetch(qs, m - kAhead);
        int sm[B], s1[B];
        v3<T> Rm[B], Am[B];
        bool any_cr = false;
        bool cr[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            sm[b] = li * B + b < n ? checked(s_cur[b]) : -1;
            s1[b] = s_next[b];
            s_next[b] = sm[b];
            if (SW || m == 0)
                bad_row |= sm[b] >= 0 ? (s1[b] >= 0 ? (s1[b] < sm[b] - 1 || s1[b] > sm[b] + 1)
                                                    : (sm[b] > 1 && sm[b] < n - 2))
                                      : (s1[b] > 0 && s1[b] < n - 1);
        }
        // SW: the anchors of the springs destroyed in step m are the log's
        // last entries, in slot order
        v3<T> dA[B];
        if constexpr (SW) {
            bool gone[B], any = false;
#pragma unroll
            for (int b = 0; b < B; ++b) {
                gone[b] = sm[b] >= 0 && s1[b] < 0;
                dA[b] = zero3<T>();
                any |= gone[b];
            }
            if (__ballot(any) != 0) {
                const uint64_t below = (1ull << lane) - 1ull;
                int tot = 0, lower = 0;
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    const uint64_t mk = __ballot(gone[b]) & segm;
                    tot += __popcll(mk);
                    lower += __popcll(mk & below);
                }
                dcount -= tot;
#pragma unroll
                for (int b = 0; b < B; ++b) {
                    if (gone[b]) {
                        const int64_t q = dcount + lower;
                        if (q >= 0 && q < a.dcap)
                            dA[b] = dlog[q];
                        else
                            bad_row = true;
                        ++lower;
                    }
                }
            }
        }
#pragma unroll
        for (int b = 0; b < B; ++b) {
            Rm[b] = R_cur[b];
            cr[b] = sm[b] < 0 && s1[b] >= 0;
            any_cr |= cr[b];
            Am[b] = zero3<T>();
            if (sm[b] >= 0) {
                v3<double> Ap = Ac[b];
                if (s1[b] < 0) {  // destroyed in step m: its advected anchor, stored by the forward or replay
                    const v3<T> v = SW ? dA[b] : trajA[(int64_t)(m + 1) * a.total + off + li * B + b];
                    Ap = {(double)v.x, (double)v.y, (double)v.z};
                }
                const v3<T> At = {T(Ap.x), T(Ap.y), T(Ap.z)};
                Ac[b] = {Ap.x + (double)(dinv[0] * At.x + dinv[1] * At.y + dinv[2] * At.z),
                         Ap.y + (double)(dinv[3] * At.x + dinv[4] * At.y + dinv[5] * At.z),
                         Ap.z + (double)(dinv[6] * At.x + dinv[7] * At.y + dinv[8] * At.z)};
                Am[b] = {T(Ac[b].x), T(Ac[b].y), T(Ac[b].z)};
            }
        }
        // created springs: their anchor depends on the end bead after the move
        if (__ballot(any_cr) != 0) {
#pragma unroll
            for (int b = 0; b < B; ++b) {
                if (cr[b]) {
                    const v3<T> g = normals3<T>(draw(kAnchor, (uint32_t)(li * B + b), gid, a.rec_g0 + mg, a.ph.key0,
                                                     a.ph.key1));
                    Gns += (double)dot(lA[b], g) * dsig;
                }
            }
#pragma unroll
            for (int bb = 0; bb < B; ++bb) {
                uint64_t mask = __ballot(cr[bb]);
                while (mask) {
                    const int L = __builtin_ctzll(mask);
                    mask &= mask - 1;
                    const int e = __builtin_amdgcn_readlane(s1[bb], L);
                    const v3<T> v = {lane_value(lA[bb].x, L), lane_value(lA[bb].y, L), lane_value(lA[bb].z, L)};
                    const int tl = (L / W) * W + e / B;
#pragma unroll
                    for (int b = 0; b < B; ++b)
                        if (lane == tl && b == e % B) lR[b] = lR[b] + v;
                }
            }
        }
        // springs per bead at step m (integer LDS atomics: order-free)
#pragma unroll
        for (int b = 0; b < B; ++b) cnt[lbase + li * B + b] = 0u;
        wave_sync();
#pragma unroll
        for (int b = 0; b < B; ++b)
            if (sm[b] >= 0) atomicAdd(&cnt[lbase + sm[b]], 1u);
        wave_sync();
        int c[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            c[b] = (int)cnt[lbase + li * B + b];
            AdjRec<T> r;
            r.v[0] = lR[b].x;
            r.v[1] = lR[b].y;
            r.v[2] = lR[b].z;
            r.v[3] = Rm[b].x;
            r.v[4] = Rm[b].y;
            r.v[5] = Rm[b].z;
            r.v[6] = T(0);
            r.v[7] = T(0);
            rec[lbase + li * B + b] = r;
        }
        wave_sync();
        // slots
        v3<T> nA[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int t = sm[b] > 0 ? sm[b] : 0;
            const AdjRec<T> r = rec[lbase + t];
            const v3<T> lRS = {r.v[0], r.v[1], r.v[2]};
            const v3<T> RS = {r.v[3], r.v[4], r.v[5]};
            nA[b] = zero3<T>();
            if (sm[b] >= 0) {
                const v3<T> dd = RS - Am[b];
                Gnsp += lRS.x * dd.x + lRS.y * dd.y + lRS.z * dd.z;
                if (s1[b] >= 0) {
                    nA[b] = lA[b] + dt * kT(kap, lA[b]);
                    const T la[3] = {lA[b].x, lA[b].y, lA[b].z};
                    const T am[3] = {Am[b].x, Am[b].y, Am[b].z};
#pragma unroll
                    for (int p = 0; p < 3; ++p)
#pragma unroll
                        for (int q = 0; q < 3; ++q) Gp[3 * p + q] += la[p] * am[q];
                }
                nA[b] = nA[b] + (dt * ks) * lRS;
            }
        }
        // beads
        const v3<T> nxt = from_next3(lR[0]);
        const v3<T> prv = from_prev3(lR[B - 1]);
        v3<T> nR[B];
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int i = li * B + b;
            const v3<T> right = (b + 1 < B) ? lR[b + 1 < B ? b + 1 : b] : nxt;
            const v3<T> left = (b > 0) ? lR[b > 0 ? b - 1 : 0] : prv;
            v3<T> lap = zero3<T>();
            if (i < n - 1) lap = lap + T(3) * (right - lR[b]);
            if (i > 0) lap = lap - T(3) * (lR[b] - left);
            if (i < n) {
                const T lr[3] = {lR[b].x, lR[b].y, lR[b].z};
                const T rm[3] = {Rm[b].x, Rm[b].y, Rm[b].z};
#pragma unroll
                for (int p = 0; p < 3; ++p)
#pragma unroll
                    for (int q = 0; q < 3; ++q) Gp[3 * p + q] += lr[p] * rm[q];
                nR[b] = lR[b] + dt * (lap - (ks * T(c[b])) * lR[b] + kT(kap, lR[b]));
            } else {
                nR[b] = zero3<T>();
            }
        }
#pragma unroll
        for (int b = 0; b < B; ++b) {
            lR[b] = nR[b];
            lA[b] = nA[b];
        }
        if (++in_block == kBlock || m == 0) {  // wave-uniform
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                G[q] += ddt * (double)Gp[q];
                Gp[q] = T(0);
            }
            Gns += kns * (double)Gnsp;
            Gnsp = T(0);
            in_block = 0;
        }
        // row m - kAhead into this step's ring slot, issued after the last
        // use of row m, so that the load can reuse its registers
        if constexpr (qs != kAhead - 1) prefetch(qs, m - kAhead);
        wave_sync();
    };
    static_assert(kAhead == 3, "the loop below is unrolled over a ring of three rows");
    int m = a.len - 1;
    for (; m >= 2; m -= 3) {  // rows m, m - 1, m - 2 in ring slots 0, 1, 2
        step_back(m, std::integral_constant<int, 0>{});
        step_back(m - 1, std::integral_constant<int, 1>{});
        step_back(m - 2, std::integral_constant<int, 2>{});
    }
    if (m >= 0) step_back(m, std::integral_constant<int, 0>{});
    if (m >= 1) step_back(m - 1, std::integral_constant<int, 1>{});

    // N_s dependence of the sampled initial anchors A = R_S + sqrt(N_s/3) g
    if (a.init_terms) {
#pragma unroll
        for (int b = 0; b < B; ++b) {
            const int j = li * B + b;
            const int s0 = (j < n) ? row_at(0, j) : -1;
            if (s0 >= 0) {
                const v3<double> g = normals3_f64(draw(kInitAnchor, (uint32_t)j, gid, 0, a.ph.key0, a.ph.key1));
                Gns += ((double)lA[b].x * g.x + (double)lA[b].y * g.y + (double)lA[b].z * g.z) * dsig;
            }
        }
    }

#pragma unroll
    for (int b = 0; b < B; ++b) {
        const int i = li * B + b;
        if (i < n) {
            T* p = lam + (off + i) * 6;
            p[0] = lR[b].x;
            p[1] = lR[b].y;
            p[2] = lR[b].z;
            p[3] = lA[b].x;
            p[4] = lA[b].y;
            p[5] = lA[b].z;
        }
    }
    if constexpr (SW) bad_row |= dcount != 0;  // every logged destruction consumed
    if (bad_row) atomicOr(a.flags, kFlagReplay);
    // per-chain sums of the lane accumulators, in lane order
#pragma unroll
    for (int q = 0; q < 9; ++q) sums[lane * 10 + q] = G[q];
    sums[lane * 10 + 9] = Gns;
    wave_sync();
    for (int v = li; v < 10; v += W) {
        double tot = 0.0;
        for (int r = 0; r < W; ++r) tot += sums[(sb + r) * 10 + v];
        if (valid) a.grad[(int64_t)chain * 10 + v] += tot;
    }
}

template <typename T, int W, int B> hipError_t launch_t(const AdjointArgs& a, hipStream_t s)
{
    constexpr int kChainsPerGroup = kWavesPerGroup * (kWaveSize / W);
    const int64_t groups = (a.n_tasks + kChainsPerGroup - 1) / kChainsPerGroup;
    if (groups == 0) return hipSuccess;
    if (a.stored)
        hipLaunchKernelGGL((k_adjoint<T, W, B, true>), dim3((unsigned)groups), dim3(kGroupThreads), 0, s, a);
    else
        hipLaunchKernelGGL((k_adjoint<T, W, B, false>), dim3((unsigned)groups), dim3(kGroupThreads), 0, s, a);
    return hipGetLastError();
}

template <typename T> hipError_t launch_p(int W, int B, const AdjointArgs& a, hipStream_t s)
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

// Byte copy (state checkpoints) in 16-byte words; sizes are multiples of 256.
__global__ void k_copy16(uint4* dst, const uint4* src, int64_t n16)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n16) dst[i] = src[i];
}

__global__ void k_rec_s0(const int32_t* S, int8_t* rec, int64_t total)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < total) rec[i] = (int8_t)S[i];
}

__global__ void k_set_ctrl_steps(int64_t* ctrl, int64_t steps)
{
    if (threadIdx.x == 0) ctrl[kCtrlSteps] = steps;
}

}  // namespace

// Scratch of the allocation-free reverse pass (ssp_adjoint_elements_noalloc):
// the per-chain gradients [kNoAllocMaxChains][10] FP64 that the element means
// are reduced from.  Every GPU the library runs on holds one copy (20 MiB)
// until the process ends; all calls on a GPU share it.  Host code never passes
// the array's name to a kernel: it is a host-side stand-in, and the device
// address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) double scratch[kNoAllocMaxChains * 10];

namespace {
std::mutex g_scratch_mu;
std::vector<double*> g_scratch_ptr;  // per device, null until looked up
}  // namespace

hipError_t noalloc_scratch(int device, double** ptr)
{
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (device < 0) return hipErrorInvalidDevice;
    if ((size_t)device >= g_scratch_ptr.size()) g_scratch_ptr.resize((size_t)device + 1, nullptr);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device) return hipErrorInvalidDevice;  // the device must be current
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = static_cast<double*>(p);
    }
    *ptr = g_scratch_ptr[device];
    return hipSuccess;
}

hipError_t launch_adjoint(int precision, int W, int B, const AdjointArgs& a, hipStream_t s)
{
    return precision == 0 ? launch_p<float>(W, B, a, s) : launch_p<double>(W, B, a, s);
}

hipError_t launch_copy_bytes(void* dst, const void* src, size_t bytes, hipStream_t s)
{
    const int64_t n16 = (int64_t)(bytes / 16);
    if (n16 == 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy16, dim3((unsigned)((n16 + 255) / 256)), dim3(256), 0, s, reinterpret_cast<uint4*>(dst),
                       reinterpret_cast<const uint4*>(src), n16);
    return hipGetLastError();
}

hipError_t launch_rec_s0(const int32_t* S, int8_t* rec, int64_t total, hipStream_t s)
{
    hipLaunchKernelGGL(k_rec_s0, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, S, rec, total);
    return hipGetLastError();
}

hipError_t launch_set_ctrl_steps(int64_t* ctrl, int64_t steps, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_ctrl_steps, dim3(1), dim3(64), 0, s, ctrl, steps);
    return hipGetLastError();
}

}  // namespace ssp
