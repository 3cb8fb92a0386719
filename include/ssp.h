/*
 * ssp.h -- C ABI of libssp, an MI355X (gfx950) library that steps large
 * ensembles of independent single-chain slip-spring chains (Uneyama,
 * "Single Chain Slip-Spring Model for Fast Rheology Simulations of Entangled
 * Polymers on GPU") and reduces their stress into the relaxation modulus G(t)
 * and per-element viscosity growth.
 *
 * Model (units b = kBT = zeta = 1, Sec. 3.1):
 *   free energy  F = sum_i 3/2 (R_{i+1}-R_i)^2 + sum_j 3/(2 N_s) (R_{S_j}-A_j)^2
 *                (Sec. 2.1, free-energy equation);
 *   Langevin     dR_i/dt = -dJ/dR_i + kappa.R_i + xi_i, dA_j/dt = kappa.A_j
 *                (Sec. 2.2), integrated by the three-substep Euler scheme of
 *                Sec. 3.1: Euler-Maruyama move, slip-spring hop, then
 *                construction/destruction at the chain ends with K = C - Z
 *                attempts (Sec. 3.2);
 *   stress       sigma = sum_i 3 b_i b_i - N 1 (Sec. 2.1 stress equation),
 *                virtual stress sigma^v = sum_j (3/N_s) d_j d_j - Z 1 with
 *                d_j = R_{S_j} - A_j (Appendix B);
 *   modulus      G(t) = <sigma(t) [sigma(0) + sigma^v(0)]> per chain in kBT
 *                units (Sec. 2.3, Green-Kubo form of the relaxation modulus).
 *
 * Conventions shared by every entry point:
 *  - Every function returns 0 on success or a negative SSP_E* code.  No C++
 *    exception crosses the ABI.  ssp_last_error() gives a message for the
 *    last failure on a handle (or, with NULL, the last failure of
 *    ssp_create/ssp_query_sizes on the calling thread).
 *  - Pointers named *_dev are device pointers on the GPU current at
 *    ssp_create; *_host are host pointers.  The caller owns every buffer;
 *    the library never frees caller memory.
 *  - Work is enqueued on the caller's stream and returns without waiting,
 *    except where a function says it synchronises.  Stream 0 (the null
 *    stream) is accepted.
 *  - A handle is not thread-safe.  Separate handles are independent.
 *  - Chains are numbered 0..n_chains-1 and grouped by element: the chains of
 *    element e are [element_offsets[e], element_offsets[e+1]).
 *  - Bead i (0-based) of chain k and slot j of chain k are entry off_k + i
 *    (resp. off_k + j) of the canonical state view, off_k = sum_{k'<k} N_k'.
 *    Slot capacity C = N per chain, one slot per bead (Sec. 3.2).
 */
#ifndef SSP_H
#define SSP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SSP_OK 0
#define SSP_EINVAL (-1)      /* invalid argument or configuration */
#define SSP_ESIZE (-2)       /* buffer too small or size overflow */
#define SSP_EHIP (-3)        /* a HIP runtime call failed */
#define SSP_ENONFINITE (-4)  /* a non-finite bead position was produced */
#define SSP_ESTATE (-5)      /* call made in the wrong order */

#define SSP_FP32 0 /* FP32 dynamics with compensated (hi, lo) position sums; FP64 stress */
#define SSP_FP64 1 /* FP64 throughout */

#define SSP_MAX_BEADS 128

typedef struct ssp_handle ssp_handle;
typedef void* ssp_stream; /* a hipStream_t */

typedef struct ssp_config {
    int64_t n_chains;               /* M >= 1 */
    int32_t n_elements;             /* E >= 1 */
    int32_t precision;              /* SSP_FP32 or SSP_FP64 */
    const int32_t* n_beads_host;    /* [M], 2 <= N_k <= SSP_MAX_BEADS; NULL: all equal to n_beads */
    int32_t n_beads;                /* N used when n_beads_host is NULL */
    int32_t sample_every;           /* n_s >= 1: stress sampled after every n_s-th step */
    const int32_t* element_offsets_host; /* [E+1], 0 = off[0] < ... <= off[E] = M; NULL: equal split */
    const int64_t* chain_ids_host;  /* [M] global chain ids keying the random streams; NULL: 0..M-1 */
    double dt;                      /* time step, > 0 (Sec. 3.1) */
    double n0;                      /* N_0: <Z>_eq = N/N_0, > 0 (Sec. 2.1) */
    double ns;                      /* N_s: slip-spring strength, > 0 (Sec. 2.1) */
    double zeta_s;                  /* slip-spring friction, > 0 (Sec. 2.2) */
    uint64_t seed;                  /* Philox key */
    int32_t max_steps_per_launch;   /* steps per kernel launch inside ssp_step; 0 = automatic */
    int32_t corr_levels;            /* multiple-tau levels (0 disables the correlator), <= 16 */
    int32_t corr_lags;              /* lags per level; must be 16 when the correlator is on */
    int32_t corr_batches;           /* chain groups for batch-means errors, 1..64 */
    int64_t series_capacity;        /* samples kept per element (0 disables the element series) */
    int32_t use_graph;              /* 1: ssp_step replays a captured hipGraph; 0: plain launches */
    int32_t construct_rule;         /* slip-spring construction attempts per step (Sec. 3.2):
                                       0 = K = C - Z (every empty slot attempts once, the GPU rule),
                                       1 = K = 1 (one attempt, by the lowest empty slot: the CPU rule) */
    int32_t corr_virtual;           /* 1: the correlator also accumulates <sigma^v(t) [sigma + sigma^v](0)>
                                       (ssp_read_correlator_virtual); 0: off */
    int32_t reserved[5];
} ssp_config;

/* Fills *cfg with the paper's standard parameters (Sec. 4.1): N_0 = 4,
 * N_s = 0.5, zeta_s = 0.1, dt = 0.01, plus n_chains = 1, n_elements = 1,
 * n_beads = 8, precision FP32, sample_every = 1, seed = 1, corr_levels 16,
 * corr_lags 16, corr_batches 16, series_capacity 0, use_graph 1,
 * construct_rule 0, corr_virtual 0. */
int ssp_config_init(ssp_config* cfg);

/* Bytes the caller must allocate on the device for the state and the work
 * buffer of *cfg.  Both must be 256-byte aligned.  Fails with SSP_EINVAL on
 * an invalid configuration (message via ssp_last_error(NULL)). */
int ssp_query_sizes(const ssp_config* cfg, size_t* state_bytes, size_t* work_bytes);

/* Validates *cfg, copies its host tables into work_dev (synchronously, on
 * the null stream), and returns a handle.  state_dev/work_dev must stay
 * allocated until ssp_destroy; the handle owns only host-side metadata,
 * compiled graphs and one internal capture stream.  The step counter starts
 * at 0. */
int ssp_create(const ssp_config* cfg, void* state_dev, void* work_dev, ssp_handle** out);

/* Samples the equilibrium initial state of every chain (Sec. 3.1, sampling
 * procedure): Gaussian bonds of variance 1/3 per component with R_0 = 0,
 * Z from Poisson(N/N_0) truncated to 0..N, S uniform on the beads, anchors
 * Gaussian about R_S with variance N_s/3 per component.  Resets the step
 * counter, the correlator and the element series. */
int ssp_init_equilibrium(ssp_handle* h, ssp_stream stream);

/* Advances every chain by n_steps >= 0 steps of the three-substep scheme
 * (Sec. 3.1) under the velocity gradient kappa_dev: [E][9] row-major FP64,
 * (kappa.R)_a = sum_b kappa[e][3a+b] R_b, constant over the call (a step
 * strain gamma is ssp_step(h, 1, gamma/dt in xy) followed by kappa = 0);
 * NULL: at rest (kappa = 0 everywhere, by a kernel variant without the flow
 * terms; the trajectory equals that of a zero table bit for bit).
 * Stress is sampled after every step whose 1-based count is a multiple of
 * sample_every; samples feed the correlator and the element series.
 * Asynchronous.  A non-finite position latches a device flag reported by the
 * next ssp_read_* call. */
int ssp_step(ssp_handle* h, int64_t n_steps, const double* kappa_dev, ssp_stream stream);

/* Per-chain stress of the current state, out_dev: [M][12] FP64 = sigma
 * (xx, yy, zz, xy, yz, zx) then sigma^v in the same order (Sec. 2.1 stress
 * equation; Appendix B virtual stress).  Synchronises the stream; returns
 * SSP_ENONFINITE if the non-finite flag is set. */
int ssp_read_stress(ssp_handle* h, double* out_dev, ssp_stream stream);

/* Ensemble average of the stress within every fluid element, out_dev:
 * [E][12] FP64, out[e][c] = (1/M_e) sum over the chains of element e of the
 * per-chain value c of ssp_read_stress (sigma, then sigma^v; Sec. 2.1 stress
 * equation, Appendix B), Neumaier-compensated in a fixed order.  Uses the
 * handle's sample staging area, which holds nothing between steps.
 * Synchronises the stream; SSP_ENONFINITE as ssp_read_stress. */
int ssp_read_element_stress(ssp_handle* h, double* out_dev, ssp_stream stream);

/* Canonical FP64 view of the state: R_dev [sum N][3], A_dev [sum N][3]
 * (hi + lo for the FP32 path), S_dev [sum N] int32 (bead index 0..N-1, or
 * -1 for an empty slot; the anchor of an empty slot is meaningless).
 * Synchronises the stream. */
int ssp_read_state(ssp_handle* h, double* R_dev, double* A_dev, int32_t* S_dev, ssp_stream stream);

/* Overwrites the state from a canonical FP64 view (same layout as
 * ssp_read_state).  S must be -1 or in 0..N_k-1.  Does not reset counters. */
int ssp_write_state(ssp_handle* h, const double* R_dev, const double* A_dev, const int32_t* S_dev,
                    ssp_stream stream);

/* Per element e and sample t (t = 0 is the first sample after the last
 * ssp_init_equilibrium or ssp_reset_observables), out_dev[e][t][0..5] =
 * sum over the chains of e of sigma (xx, yy, zz, xy, yz, zx), summed with
 * Neumaier-compensated FP64.  The viscosity growth of a shear element is
 * out[e][t][3] / (M_e gamma_dot_e) (Sec. 4.1, viscosity growth).  out_dev
 * holds [E][series_capacity][6]; *n_samples_host receives the number of
 * valid samples (<= series_capacity).  Synchronises the stream. */
int ssp_read_element_series(ssp_handle* h, double* out_dev, int64_t* n_samples_host, ssp_stream stream);

/* Relaxation modulus from the multiple-tau correlator (Green-Kubo form,
 * Sec. 2.3): for level l and lag k, G[l][k] = mean over chains and over the
 * components xy, yz, zx of <x(t) y(t - tau)>, x = sigma_ab, y = sigma_ab +
 * sigma^v_ab, with the level-l series made of pairwise means of level l-1
 * and tau = k 2^l sample_every dt.  G_dev, G_err_dev: [levels][16] FP64
 * (G_err = batch-means standard error over corr_batches chain groups; 0 when
 * corr_batches = 1); tau_host [levels][16]; counts_host [levels][16] int64
 * number of products per chain and component (0 = no data, G = 0).  Chain
 * sums are Neumaier-compensated.  Synchronises the stream. */
int ssp_read_correlator(ssp_handle* h, double* G_dev, double* G_err_dev, double* tau_host, int64_t* counts_host,
                        ssp_stream stream);

/* The virtual-stress channel of the correlator (config corr_virtual = 1):
 * Gv(t) = <sigma^v_ab(t) [sigma_ab + sigma^v_ab](t0)> per chain in kBT units,
 * averaged over ab in {xy, yz, zx}, on the same multiple-tau grid, counts and
 * batch-means errors as ssp_read_correlator.  dGv(t) = Gv(t) / G(t) is the
 * relative contribution of the virtual stress to the shear relaxation modulus
 * of Sec. 4.1 (its numerator <sigma^v(t) sigma> + <sigma^v(t) sigma^v> over
 * the denominator <sigma(t) sigma> + <sigma(t) sigma^v>), NaN at lags without
 * data or where G = 0.  Gv_dev, Gv_err_dev, dGv_dev: [corr_levels][16] FP64
 * (device); dGv_dev may be NULL.  Synchronises the stream.  SSP_ESTATE when
 * the channel is off. */
int ssp_read_correlator_virtual(ssp_handle* h, double* Gv_dev, double* Gv_err_dev, double* dGv_dev,
                                ssp_stream stream);

/* Linear viscoelasticity from the relaxation modulus (the relations of
 * Sec. 4.1): G'(w) = w int G(t) sin(w t) dt, G''(w) = w int G(t) cos(w t) dt,
 * |eta*(w)| = |G' + i G''| / w, eta_0 = int G(t) dt, and the longest
 * relaxation time from 1/tau_d = -lim ln G(t) / t.
 * G_dev: [corr_levels][16] FP64 device array as written by ssp_read_correlator
 * (or any modulus on that grid), read on the grid of the handle's current
 * sample count: level 0 lags 0..15, level l >= 1 lags 8..15, lag times
 * k 2^l sample_every dt, lags with data only.  The integrals take G piecewise
 * linear between grid points (the trapezoidal rule's model of G) and
 * integrate that exactly against sin and cos, up to the last point with data;
 * eta_0 is the trapezoidal sum.  tau_d = -1 / (least-squares slope of ln G
 * against t over the grid points with t_lo <= t <= t_hi and G > 0); NaN with
 * fewer than two such points or a slope that is not negative.
 * omega_dev: [n_omega] angular frequencies > 0 (device); moduli_dev:
 * [n_omega][3] FP64 G', G'', |eta*| (device); scalars_dev: [2] FP64 eta_0,
 * tau_d (device).  Asynchronous.  SSP_ESTATE without a correlator;
 * SSP_EINVAL for missing buffers, n_omega < 0 or t_lo > t_hi. */
int ssp_linear_viscoelasticity(ssp_handle* h, const double* G_dev, const double* omega_dev, int32_t n_omega,
                               double t_lo, double t_hi, double* moduli_dev, double* scalars_dev, ssp_stream stream);

/* Clears the correlator and the element series; the next sample is t = 0. */
int ssp_reset_observables(ssp_handle* h, ssp_stream stream);

/* Steps completed since ssp_init_equilibrium. */
int ssp_step_count(const ssp_handle* h, int64_t* steps_host);

/* The three standard normals the Euler move of step `step` draws for bead
 * `bead` of the chain with global id `chain_id`, computed on the device in
 * the handle's precision: out_dev [count][3] FP64 for beads bead..bead+count-1.
 * Streams (Philox4x32-10, key = seed, counter = (index, chain id, k lo,
 * k hi | purpose << 24), k = step >> 1): steps 2k and 2k+1 share the Box-Muller
 * normals (a0..a5) of blocks NOISE (a0..a3) and NOISE2 (a4, a5); step 2k
 * takes (a0, a1, a2), step 2k+1 takes (a3, a4, a5).  Used to test the random
 * streams in isolation. */
int ssp_rng_normals(ssp_handle* h, int64_t chain_id, int64_t step, int32_t bead, int32_t count, double* out_dev,
                    ssp_stream stream);

/* ---- Differentiation (pathwise adjoint, conditioned on the events) --------
 * The derivative of a final stress component J_k = sigma_c(R_T) of every
 * chain k with respect to the velocity gradient kappa (all nine entries) and
 * the slip-spring strength N_s, taken through the Euler map of Sec. 3.1 with
 * the recorded hop/creation/destruction events and the random normals held
 * fixed (the dependence of the event probabilities on the parameters is not
 * included).  Created anchors A = R_end + sqrt(N_s/3) g carry their N_s
 * dependence.  Memory: (window+1) bytes per bead for the slot trajectory,
 * one state copy per checkpoint, and (ckpt_every+1) x 6 reals per bead for
 * the replay of one segment. */

/* Bytes of the caller-owned recording buffer for a window of `window` steps
 * with a checkpoint every `ckpt_every` steps.  The buffer holds the slot rows
 * ((window + 1) x total beads, 1 byte each), the checkpoints, and the
 * positions and anchors of one segment (2 (ckpt_every + 1) x total beads x 3
 * values of the path's precision).  With ckpt_every >= window (a stored
 * window) it holds instead the positions of the whole window ((window + 1) x
 * total beads x 3 values), the anchors at its end, and a per-chain log of
 * the anchors of destroyed springs sized from the creation rate: about 13 B
 * per bead-step in FP32. */
int ssp_adjoint_bytes(const ssp_handle* h, int64_t window, int32_t ckpt_every, size_t* bytes);

/* Advances the ensemble by `window` steps exactly like ssp_step (same
 * trajectory, samples and counters) while recording the slot state after every
 * step and a state checkpoint every ckpt_every steps into rec_dev (256-byte
 * aligned, ssp_adjoint_bytes long).  With ckpt_every >= window the window is
 * one segment and the forward also stores its positions and the anchors the
 * reverse pass needs, so that ssp_adjoint replays nothing (memory for time).
 * kappa_dev as in ssp_step (NULL: at rest).  Asynchronous. */
int ssp_forward_record(ssp_handle* h, int64_t window, int32_t ckpt_every, const double* kappa_dev, void* rec_dev,
                       ssp_stream stream);

/* Reverse pass over the last recorded window: for every checkpoint segment,
 * last to first, replays the segment from its checkpoint (bitwise the same
 * trajectory; a one-segment window uses the trajectory its forward stored)
 * and runs the adjoint recursion through it.  grad_dev [M][10]
 * FP64 receives dJ_k/dkappa_ab (row-major, 9 values) and dJ_k/dN_s for
 * J_k = sigma_component of chain k at the end of the window (component 0..5
 * = xx yy zz xy yz zx).  kappa_dev must hold the velocity gradient of the
 * recorded window (NULL: at rest).  init_window != 0 adds the N_s dependence of the sampled
 * initial anchors when the window started at step 0.  Synchronises.  Every
 * recorded slot row is checked as it is read (a state the step could have
 * produced from the one before); a recording changed since
 * ssp_forward_record fails with SSP_EINVAL, leaves the ensemble's own state
 * untouched and gives no valid gradients.  A stored window in which a chain
 * destroyed more springs than its log holds (far beyond the expected count)
 * fails with SSP_ESIZE; record such a window with checkpoints. */
int ssp_adjoint(ssp_handle* h, const void* rec_dev, const double* kappa_dev, int32_t component, int32_t init_window,
                double* grad_dev, ssp_stream stream);

/* The reverse pass of ssp_adjoint reduced per fluid element: elem_grad_dev
 * [E][10] FP64 receives the ensemble averages over the chains of each element
 * of dJ_k/dkappa_ab (9, row-major) and dJ_k/dN_s, i.e. the gradients of the
 * element's mean final stress component (1/M_e) sum_k sigma_component,k, each
 * a Neumaier-compensated sum in a fixed order divided by M_e.
 * chain_grad_dev [M][10] FP64 is the caller's workspace for the per-chain
 * gradients and holds them on return (as ssp_adjoint's grad_dev).  Other
 * arguments, synchronisation and errors as ssp_adjoint; on an error
 * elem_grad_dev is not written. */
int ssp_adjoint_elements(ssp_handle* h, const void* rec_dev, const double* kappa_dev, int32_t component,
                         int32_t init_window, double* chain_grad_dev, double* elem_grad_dev, ssp_stream stream);

/* ssp_adjoint_elements for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same element means into elem_grad_dev [E][10] FP64, with
 * the per-chain gradients kept in a static device array of the library
 * instead of a caller workspace.  Allocates nothing and calls no allocating
 * routine.  At most 262144 chains (SSP_ESIZE beyond).  The array (20 MiB per
 * GPU, held until the process ends) is shared by every handle on a GPU, so
 * calls that overlap on one GPU race; it keeps the last call's contents, and
 * each call clears what it uses.  Other arguments, synchronisation and errors
 * as ssp_adjoint_elements. */
int ssp_adjoint_elements_noalloc(ssp_handle* h, const void* rec_dev, const double* kappa_dev, int32_t component,
                                 int32_t init_window, double* elem_grad_dev, ssp_stream stream);

/* Chain-to-wavefront mapping for the chains with n_lo <= N <= n_hi: each
 * such chain occupies lanes_per_chain lanes (8, 16, 32 or 64) with
 * beads_per_lane beads and slots per lane (1, or 2 with 16, 32 or 64 lanes);
 * lanes_per_chain * beads_per_lane >= n_hi.  Trajectories do not depend on the
 * mapping (each bead's arithmetic is the same); FP64 stress sums may differ in
 * the last bits.  The default is the narrowest one-bead-per-lane segment that
 * fits (two beads per lane for N > 64).  Synchronises the device; drops
 * captured graphs.  Used by the autotuner. */
int ssp_set_mapping(ssp_handle* h, int32_t n_lo, int32_t n_hi, int32_t lanes_per_chain, int32_t beads_per_lane);

/* Launch schedule of the step kernel for ssp_step (the recorded and stored
 * forwards keep the plain one).  persistent != 0 (the default): as many
 * workgroups as fit on the device run the launch's steps as units of (time
 * chunk, wavefront's chains), taken from a queue in the work buffer, a unit
 * starting once the previous chunk of the same chains has stored their
 * state, so that no partly filled last round of wavefronts is left; 0: one
 * wavefront per group of chains for the whole launch.  Trajectories are the
 * same bit for bit.  Synchronises the device; drops captured graphs. */
int ssp_set_schedule(ssp_handle* h, int persistent);

/* Kernel timing mode (for measurement): while enabled, ssp_step launches
 * without a graph and brackets the step-kernel launches of every chunk with
 * hipEvents on the caller's stream. */
int ssp_set_kernel_timing(ssp_handle* h, int enable);

/* Synchronises the recorded events and returns the summed step-kernel time in
 * ms, the number of timed chunks and the bead-steps they covered since the
 * previous call; then clears the totals. */
int ssp_kernel_time(ssp_handle* h, double* ms_host, int64_t* launches_host, int64_t* bead_steps_host);

/* Releases host resources (graphs, capture stream).  Caller memory untouched. */
int ssp_destroy(ssp_handle* h);

/* Message for the last error on h (NULL: last create/query error). */
const char* ssp_last_error(const ssp_handle* h);

/* Warning about a configuration that is accepted but leaves the regime the
 * step map of Sec. 3.1 is written for, or NULL when there is none: with
 * dt / zeta_s > 1/4 the 1/2 caps on the hop probabilities can bind (and, for
 * larger ratios, those on construction and destruction), so the step no
 * longer follows the continuous-time hop rates it discretises.  h: the
 * handle's configuration; NULL: the configuration of the last ssp_query_sizes
 * or ssp_create on the calling thread.  The string is owned by the library. */
const char* ssp_warning(const ssp_handle* h);

#ifdef __cplusplus
}
#endif

#endif /* SSP_H */
