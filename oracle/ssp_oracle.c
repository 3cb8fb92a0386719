/*
 * ssp_oracle.c -- plain FP64 CPU oracle for the single-chain slip-spring
 * ensemble (Uneyama, "Single Chain Slip-Spring Model for Fast Rheology
 * Simulations of Entangled Polymers on GPU").
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may include, link,
 * load or call this file: it exists so that tests, the smoke check and the
 * benchmark's CPU-baseline leg can check the HIP library against an
 * independent, obviously-correct implementation.  It shares no code, header,
 * table or constant generator with the HIP path.
 *
 * Everything is double precision, written as scalar loops in the order the
 * paper states the method.  Units: b = kBT = zeta = 1 (Sec. 3.1), so the bond
 * stiffness 3 kBT/b^2 is 3 and the slip-spring stiffness is 3/N_s.
 *
 * Indexing: beads i = 0..N-1 (the paper's 1..N), slip-spring slots
 * j = 0..N-1.  A slot holds S_j in 0..N-1 when occupied and -1 when empty.
 * Chain k occupies entries [off[k], off[k] + N[k]) of the bead arrays and of
 * the slot arrays (slot capacity C = N, one slot per bead, Sec. 3.2).
 * Positions are stored as xyz triples: R[3*(off+i)+a].
 *
 * Readings of the paper taken here (each is listed with its reason in the
 * design notes of the repository):
 *  - Euler step: R(t+dt) = R(t) + dt(-dJ/dR + kappa.R) + sqrt(2 dt) w, and
 *    A(t+dt) = A(t) + dt kappa.A (the printed update drops the R(t), A(t)
 *    terms; only this reading integrates the Langevin equation, Sec. 2.2).
 *  - Hop (Sec. 3.1, substep 2): one uniform u per spring; S+1 if u < P+,
 *    else S-1 if u < P+ + P-.  Positions used are the post-Langevin ones.
 *  - Reconstruction (Sec. 3.1 substep 3 with K = C - Z attempts, Sec. 3.2):
 *    every empty slot makes one attempt from the post-hop state with
 *    p = min(dt/(zeta_s N0 K), 1/2) at bead 0 and p at bead N-1 (one
 *    uniform: [0,p) -> bead 0, [p,2p) -> bead N-1).  Occupied slots sitting
 *    on an end are destroyed with min(dt/zeta_s (delta_{S,0}+delta_{S,N-1}), 1).
 *    A spring created in this step is not tested for destruction.  The CPU
 *    rule K = 1 of Sec. 3.2 is a variant: only the lowest empty slot attempts,
 *    with p = min(dt/(zeta_s N0), 1/2).
 *  - Virtual stress sums over all Z springs (Appendix B form).
 *  - Initial Z is drawn from Poisson(N/N0) truncated to 0..C.
 *
 * Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11,
 * "Parallel random numbers: as easy as 1, 2, 3"), implemented here from the
 * published round function.  key = (seed_lo, seed_hi); counter =
 * (index, chain_id, step_lo, step_hi | purpose << 24), steps below 2^56.
 * A 32-bit word w maps to u = ((w >> 9) + 0.5) * 2^-23 in (0,1); normals
 * come from the Box-Muller transform r = sqrt(-2 ln u_a), theta = 2 pi u_b,
 * (r cos theta, r sin theta).  Three normals per block: the pair from
 * (w0,w1) and the cosine member of the pair from (w2,w3).
 *
 * Per-step streams come in step pairs (2k, 2k+1), three blocks per bead or
 * slot index and pair, all with counter step word k:
 *   NOISE(i, k)  = x: Box-Muller pairs (x0,x1) -> (a0, a1), (x2,x3) -> (a2, a3);
 *   NOISE2(i, k) = y: Box-Muller pair (y0,y1) -> (a4, a5); y2, y3 are the hop
 *                  and reconstruction words of slot i at step 2k;
 *   SLOT(j, k)   = z: z0, z1 are the hop and reconstruction words of slot j at
 *                  step 2k+1 (z2, z3 unused).
 * The bead noise is (a0, a1, a2) at step 2k and (a3, a4, a5) at step 2k+1.
 * Six normals and four uniforms per pair take 1.5 blocks per step.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Threads the OpenMP loops over chains use. */
int ssp_oracle_threads(void) { return omp_get_max_threads(); }

/* Threads of the later parallel loops (the benchmark times the oracle on one
 * thread and on all of them). */
void ssp_oracle_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

/* ---- Philox4x32-10, from the published definition ---------------------- */

#define PHILOX_M0 0xD2511F53u
#define PHILOX_M1 0xCD9E8D57u
#define PHILOX_W0 0x9E3779B9u
#define PHILOX_W1 0xBB67AE85u

enum {
    P_INIT_BOND = 1,
    P_INIT_Z = 2,
    P_INIT_S = 3,
    P_INIT_ANCHOR = 4,
    P_NOISE = 5,
    P_SLOT = 6,
    P_ANCHOR = 7,
    P_NOISE2 = 8
};

void ssp_oracle_philox(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {
            k0 += PHILOX_W0;
            k1 += PHILOX_W1;
        }
        uint64_t p0 = (uint64_t)PHILOX_M0 * (uint64_t)c0;
        uint64_t p1 = (uint64_t)PHILOX_M1 * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

static void draw(uint64_t seed, int purpose, int index, int64_t chain, int64_t step, uint32_t w[4])
{
    uint32_t ctr[4], key[2];
    ctr[0] = (uint32_t)index;
    ctr[1] = (uint32_t)chain;
    ctr[2] = (uint32_t)((uint64_t)step & 0xffffffffu);
    ctr[3] = (uint32_t)((uint64_t)step >> 32) | ((uint32_t)purpose << 24);
    key[0] = (uint32_t)(seed & 0xffffffffu);
    key[1] = (uint32_t)(seed >> 32);
    ssp_oracle_philox(ctr, key, w);
}

double ssp_oracle_u01(uint32_t w)
{
    return ((double)(w >> 9) + 0.5) * (1.0 / 8388608.0);
}

/* Three standard normals from one Philox block. */
static void normals3(const uint32_t w[4], double n[3])
{
    double r1 = sqrt(-2.0 * log(ssp_oracle_u01(w[0])));
    double t1 = 2.0 * M_PI * ssp_oracle_u01(w[1]);
    double r2 = sqrt(-2.0 * log(ssp_oracle_u01(w[2])));
    double t2 = 2.0 * M_PI * ssp_oracle_u01(w[3]);
    n[0] = r1 * cos(t1);
    n[1] = r1 * sin(t1);
    n[2] = r2 * cos(t2);
}

void ssp_oracle_normals3(uint64_t seed, int purpose, int index, int64_t chain, int64_t step, double n[3])
{
    uint32_t w[4];
    draw(seed, purpose, index, chain, step, w);
    normals3(w, n);
}

void ssp_oracle_block(uint64_t seed, int purpose, int index, int64_t chain, int64_t step, uint32_t w[4])
{
    draw(seed, purpose, index, chain, step, w);
}

/* The Box-Muller pair (r cos t, r sin t) of two words. */
static void box_muller(uint32_t wa, uint32_t wb, double* c, double* s)
{
    double r = sqrt(-2.0 * log(ssp_oracle_u01(wa)));
    double t = 2.0 * M_PI * ssp_oracle_u01(wb);
    *c = r * cos(t);
    *s = r * sin(t);
}

/* Noise normals of bead i of chain c at step `step` (step-pair layout above). */
void ssp_oracle_step_noise(uint64_t seed, int i, int64_t c, int64_t step, double g[3])
{
    const int64_t k = step >> 1;
    uint32_t x[4];
    double a0, a1, a2, a3;
    draw(seed, P_NOISE, i, c, k, x);
    box_muller(x[0], x[1], &a0, &a1);
    box_muller(x[2], x[3], &a2, &a3);
    if ((step & 1) == 0) {
        g[0] = a0;
        g[1] = a1;
        g[2] = a2;
    } else {
        uint32_t y[4];
        double a4, a5;
        draw(seed, P_NOISE2, i, c, k, y);
        box_muller(y[0], y[1], &a4, &a5);
        g[0] = a3;
        g[1] = a4;
        g[2] = a5;
    }
}

/* Hop word w[0] and reconstruction word w[1] of slot j of chain c at step
 * `step` (step-pair layout above). */
void ssp_oracle_slot_words(uint64_t seed, int j, int64_t c, int64_t step, uint32_t w[2])
{
    uint32_t b[4];
    if ((step & 1) == 0) {
        draw(seed, P_NOISE2, j, c, step >> 1, b);
        w[0] = b[2];
        w[1] = b[3];
    } else {
        draw(seed, P_SLOT, j, c, step >> 1, b);
        w[0] = b[0];
        w[1] = b[1];
    }
}

/* ---- Initial equilibrium state (Sec. 3.1, sampling procedure) ------------ */

/* P_eq(Z) is Poisson with mean N/N0 (Sec. 2.1); truncated to 0..C because a
 * chain has only C slots (Sec. 3.2). */
static int sample_truncated_poisson(double lambda, int cap, double u)
{
    double pmf = exp(-lambda);
    double total = 0.0;
    double* cdf = (double*)malloc(sizeof(double) * (size_t)(cap + 1));
    for (int z = 0; z <= cap; ++z) {
        if (z > 0) pmf = pmf * lambda / (double)z;
        total += pmf;
        cdf[z] = total;
    }
    int result = cap;
    for (int z = 0; z <= cap; ++z) {
        if (u < cdf[z] / total) {
            result = z;
            break;
        }
    }
    free(cdf);
    return result;
}

void ssp_oracle_init(int n_chains, const int32_t* N, const int64_t* off, const int64_t* chain_id,
                     double n0, double ns, uint64_t seed, double* R, double* A, int32_t* S)
{
    const double bond_sd = sqrt(1.0 / 3.0);   /* bond variance b^2/3 per component */
    const double anchor_sd = sqrt(ns / 3.0);  /* anchor variance N_s b^2/3 per component */
#pragma omp parallel for schedule(dynamic, 16)
    for (int k = 0; k < n_chains; ++k) {
        const int n = N[k];
        const int64_t o = off[k];
        const int64_t c = chain_id[k];
        double* r = R + 3 * o;
        double* a = A + 3 * o;
        int32_t* s = S + o;
        /* 1. Gaussian chain: R_0 = 0, bonds N(0, 1/3). */
        r[0] = r[1] = r[2] = 0.0;
        for (int i = 0; i + 1 < n; ++i) {
            double g[3];
            ssp_oracle_normals3(seed, P_INIT_BOND, i, c, 0, g);
            for (int d = 0; d < 3; ++d) r[3 * (i + 1) + d] = r[3 * i + d] + bond_sd * g[d];
        }
        /* 2. Z from the (truncated) Poisson distribution. */
        uint32_t w[4];
        draw(seed, P_INIT_Z, 0, c, 0, w);
        int z = sample_truncated_poisson((double)n / n0, n, ssp_oracle_u01(w[0]));
        /* 3. Slots 0..Z-1: S uniform on the beads, anchor Gaussian about R_S. */
        for (int j = 0; j < n; ++j) {
            if (j < z) {
                draw(seed, P_INIT_S, j, c, 0, w);
                int sj = (int)(((uint64_t)w[0] * (uint64_t)n) >> 32);
                double g[3];
                ssp_oracle_normals3(seed, P_INIT_ANCHOR, j, c, 0, g);
                s[j] = sj;
                for (int d = 0; d < 3; ++d) a[3 * j + d] = r[3 * sj + d] + anchor_sd * g[d];
            } else {
                s[j] = -1;
                a[3 * j] = a[3 * j + 1] = a[3 * j + 2] = 0.0;
            }
        }
    }
}

/* Discrete hop probability of a spring on bead i with anchor aj toward bead
 * i + dir (dir = +1 or -1): min{(dt/zeta_s)[1 - tanh(3/(4 N_s) ((R_{i+dir} -
 * A)^2 - (R_i - A)^2))], 1/2}, and 0 when i + dir leaves the chain (Sec. 3.1,
 * substep 2, from the Glauber rates of Sec. 2.2). */
double ssp_oracle_hop_prob(int n, const double* r, const double* aj, int i, int dir, double dt, double ns,
                           double zeta_s)
{
    int t = i + dir;
    if (t < 0 || t > n - 1) return 0.0;
    double d0 = 0.0, d1 = 0.0;
    for (int d = 0; d < 3; ++d) {
        double x0 = r[3 * i + d] - aj[d];
        double x1 = r[3 * t + d] - aj[d];
        d0 += x0 * x0;
        d1 += x1 * x1;
    }
    double p = dt / zeta_s * (1.0 - tanh(3.0 / (4.0 * ns) * (d1 - d0)));
    return p > 0.5 ? 0.5 : p;
}

/* ---- One time step (Sec. 3.1, three substeps) ---------------------------- */

/* Event bits written per slot when an event array is given. */
#define EV_HOP_UP 1
#define EV_HOP_DOWN 2
#define EV_DESTROY 4
#define EV_CREATE_FIRST 8
#define EV_CREATE_LAST 16

/* Advances every chain by one step with step index `step` (the RNG counter).
 * kappa: [n_chains][9] row-major velocity gradient per chain, (kappa.R)_a =
 * sum_b kappa[a][b] R_b.  Optional outputs (may be NULL): events[slot] bits
 * above; margin[slot] = smallest |u - threshold| over the decisions that slot
 * took in this step (1.0 when it took none). */
/* Substep 1 of Sec. 3.1 for one chain: forces F = -dJ/dR at time t (free
 * energy of Sec. 2.1) with the slot state s, then the Euler-Maruyama move of
 * the beads and the affine advection of the occupied anchors. */
static void move_chain(int n, int64_t c, const double* kap, double dt, double ns, uint64_t seed, int64_t step,
                       double* r, double* a, const int32_t* s, double* F, double* ro)
{
    const double kb = 3.0;
    const double ks = 3.0 / ns;
    const double sq2dt = sqrt(2.0 * dt);

    for (int i = 0; i < 3 * n; ++i) F[i] = 0.0;
    for (int i = 0; i < 3 * n; ++i) F[i] = 0.0;
    for (int i = 0; i + 1 < n; ++i) {
        for (int d = 0; d < 3; ++d) {
            double b = r[3 * (i + 1) + d] - r[3 * i + d];
            F[3 * i + d] += kb * b;
            F[3 * (i + 1) + d] -= kb * b;
        }
    }
    for (int j = 0; j < n; ++j) {
        if (s[j] < 0) continue;
        int i = s[j];
        for (int d = 0; d < 3; ++d) F[3 * i + d] -= ks * (r[3 * i + d] - a[3 * j + d]);
    }
    /* Euler-Maruyama for beads; advection for occupied anchors. */
    for (int i = 0; i < 3 * n; ++i) ro[i] = r[i];
    for (int i = 0; i < n; ++i) {
        double g[3];
        ssp_oracle_step_noise(seed, i, c, step, g);
        for (int d = 0; d < 3; ++d) {
            double flow = kap[3 * d + 0] * ro[3 * i + 0] + kap[3 * d + 1] * ro[3 * i + 1] + kap[3 * d + 2] * ro[3 * i + 2];
            r[3 * i + d] = ro[3 * i + d] + dt * (F[3 * i + d] + flow) + sq2dt * g[d];
        }
    }
    for (int j = 0; j < n; ++j) {
        if (s[j] < 0) continue;
        double a0 = a[3 * j], a1 = a[3 * j + 1], a2 = a[3 * j + 2];
        for (int d = 0; d < 3; ++d) {
            double flow = kap[3 * d + 0] * a0 + kap[3 * d + 1] * a1 + kap[3 * d + 2] * a2;
            a[3 * j + d] += dt * flow;
        }
    }
}

static void step_chain(int n, int64_t c, const double* kap, double dt, double n0, double ns, double zeta_s,
                       int rule, uint64_t seed, int64_t step, double* r, double* a, int32_t* s, uint8_t* ev,
                       double* margin, double* F, double* ro)
{
    const double anchor_sd = sqrt(ns / 3.0);
    const double ch = dt / zeta_s;

    if (ev)
        for (int j = 0; j < n; ++j) ev[j] = 0;
    if (margin)
        for (int j = 0; j < n; ++j) margin[j] = 1.0;

    /* Substep 1: move. */
    move_chain(n, c, kap, dt, ns, seed, step, r, a, s, F, ro);

    /* Substep 2: hops, all springs from the same post-Langevin positions. */
    uint32_t w[4];
    int32_t* s_after = (int32_t*)malloc(sizeof(int32_t) * (size_t)n);
    for (int j = 0; j < n; ++j) {
        s_after[j] = s[j];
        if (s[j] < 0) continue;
        int i = s[j];
        double pp = ssp_oracle_hop_prob(n, r, a + 3 * j, i, +1, dt, ns, zeta_s);
        double pm = ssp_oracle_hop_prob(n, r, a + 3 * j, i, -1, dt, ns, zeta_s);
        ssp_oracle_slot_words(seed, j, c, step, w);
        double u = ssp_oracle_u01(w[0]);
        if (u < pp) {
            s_after[j] = i + 1;
            if (ev) ev[j] |= EV_HOP_UP;
        } else if (u < pp + pm) {
            s_after[j] = i - 1;
            if (ev) ev[j] |= EV_HOP_DOWN;
        }
        if (margin) {
            double m = fabs(u - pp);
            double m2 = fabs(u - (pp + pm));
            if (m2 < m) m = m2;
            if (m < margin[j]) margin[j] = m;
        }
    }
    for (int j = 0; j < n; ++j) s[j] = s_after[j];
    free(s_after);

    /* Substep 3: reconstruction at the chain ends from the post-hop state.
     * Construction is attempted K times (Sec. 3.1 substep 3).  Rule 0, the GPU
     * rule of Sec. 3.2: K = C - Z, every empty slot attempts once.  Rule 1, the
     * CPU rule of Sec. 3.2: K = 1, a single attempt, made by the lowest empty
     * slot (none when all C slots are occupied). */
    int z = 0, first_empty = -1;
    for (int j = 0; j < n; ++j) {
        z += (s[j] >= 0);
        if (s[j] < 0 && first_empty < 0) first_empty = j;
    }
    int kattempt = rule == 1 ? (z < n ? 1 : 0) : n - z;
    double p = 0.0;
    if (kattempt > 0) {
        p = dt / (zeta_s * n0 * (double)kattempt);
        if (p > 0.5) p = 0.5;
    }
    for (int j = 0; j < n; ++j) {
        ssp_oracle_slot_words(seed, j, c, step, w);
        double u = ssp_oracle_u01(w[1]);
        if (s[j] >= 0) {
            int ends = (s[j] == 0) + (s[j] == n - 1);
            if (ends == 0) continue;
            double pd = ch * (double)ends;
            if (pd > 1.0) pd = 1.0;
            if (u < pd) {
                s[j] = -1;
                a[3 * j] = a[3 * j + 1] = a[3 * j + 2] = 0.0;
                if (ev) ev[j] |= EV_DESTROY;
            }
            if (margin) {
                double m = fabs(u - pd);
                if (m < margin[j]) margin[j] = m;
            }
        } else if (rule == 0 || j == first_empty) {
            int at = -1;
            if (u < p) {
                at = 0;
                if (ev) ev[j] |= EV_CREATE_FIRST;
            } else if (u < 2.0 * p) {
                at = n - 1;
                if (ev) ev[j] |= EV_CREATE_LAST;
            }
            if (margin) {
                double m = fabs(u - p);
                double m2 = fabs(u - 2.0 * p);
                if (m2 < m) m = m2;
                if (m < margin[j]) margin[j] = m;
            }
            if (at >= 0) {
                double g[3];
                ssp_oracle_normals3(seed, P_ANCHOR, j, c, step, g);
                s[j] = at;
                for (int d = 0; d < 3; ++d) a[3 * j + d] = r[3 * at + d] + anchor_sd * g[d];
            }
        }
    }
}

/* Per-chain stress sigma (Eq. for the stress operator) and virtual stress
 * sigma^v (Appendix B), 12 values: sigma xx yy zz xy yz zx, then sigma^v in the
 * same order. */
static void stress_chain(int n, double ns, const double* r, const double* a, const int32_t* s, double out[12])
{
    for (int q = 0; q < 12; ++q) out[q] = 0.0;
    for (int i = 0; i + 1 < n; ++i) {
        double b[3];
        for (int d = 0; d < 3; ++d) b[d] = r[3 * (i + 1) + d] - r[3 * i + d];
        out[0] += 3.0 * b[0] * b[0];
        out[1] += 3.0 * b[1] * b[1];
        out[2] += 3.0 * b[2] * b[2];
        out[3] += 3.0 * b[0] * b[1];
        out[4] += 3.0 * b[1] * b[2];
        out[5] += 3.0 * b[2] * b[0];
    }
    out[0] -= (double)n;
    out[1] -= (double)n;
    out[2] -= (double)n;
    int z = 0;
    for (int j = 0; j < n; ++j) {
        if (s[j] < 0) continue;
        ++z;
        double d[3];
        for (int e = 0; e < 3; ++e) d[e] = r[3 * s[j] + e] - a[3 * j + e];
        double k = 3.0 / ns;
        out[6] += k * d[0] * d[0];
        out[7] += k * d[1] * d[1];
        out[8] += k * d[2] * d[2];
        out[9] += k * d[0] * d[1];
        out[10] += k * d[1] * d[2];
        out[11] += k * d[2] * d[0];
    }
    out[6] -= (double)z;
    out[7] -= (double)z;
    out[8] -= (double)z;
}

void ssp_oracle_stress(int n_chains, const int32_t* N, const int64_t* off, double ns, const double* R,
                       const double* A, const int32_t* S, double* out)
{
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n_chains; ++k) {
        int64_t o = off[k];
        stress_chain(N[k], ns, R + 3 * o, A + 3 * o, S + o, out + 12 * (int64_t)k);
    }
}

/* One step for all chains.  events/margin may be NULL. */
void ssp_oracle_step(int n_chains, const int32_t* N, const int64_t* off, const int64_t* chain_id,
                     const double* kappa, double dt, double n0, double ns, double zeta_s, int rule, uint64_t seed,
                     int64_t step, double* R, double* A, int32_t* S, uint8_t* events, double* margin)
{
#pragma omp parallel for schedule(dynamic, 8)
    for (int k = 0; k < n_chains; ++k) {
        int n = N[k];
        int64_t o = off[k];
        double* F = (double*)malloc(sizeof(double) * 3 * (size_t)n);
        double* ro = (double*)malloc(sizeof(double) * 3 * (size_t)n);
        step_chain(n, chain_id[k], kappa + 9 * (int64_t)k, dt, n0, ns, zeta_s, rule, seed, step, R + 3 * o,
                   A + 3 * o, S + o, events ? events + o : NULL, margin ? margin + o : NULL, F, ro);
        free(F);
        free(ro);
    }
}

/* n_steps steps starting at step index step0, sampling the 12 stress values of
 * every chain after each step whose 1-based count (step + 1) is a multiple of
 * sample_every.  samples: [n_samples][n_chains][12] (may be NULL).  Returns
 * the number of samples written. */
int64_t ssp_oracle_run(int n_chains, const int32_t* N, const int64_t* off, const int64_t* chain_id,
                       const double* kappa, double dt, double n0, double ns, double zeta_s, int rule, uint64_t seed,
                       int64_t step0, int64_t n_steps, int64_t sample_every, double* R, double* A, int32_t* S,
                       double* samples)
{
    int64_t n_samples = 0;
    for (int64_t t = step0; t < step0 + n_steps; ++t)
        if ((t + 1) % sample_every == 0) ++n_samples;
#pragma omp parallel for schedule(dynamic, 4)
    for (int k = 0; k < n_chains; ++k) {
        int n = N[k];
        int64_t o = off[k];
        double* F = (double*)malloc(sizeof(double) * 3 * (size_t)n);
        double* ro = (double*)malloc(sizeof(double) * 3 * (size_t)n);
        int64_t q = 0;
        for (int64_t t = step0; t < step0 + n_steps; ++t) {
            step_chain(n, chain_id[k], kappa + 9 * (int64_t)k, dt, n0, ns, zeta_s, rule, seed, t, R + 3 * o,
                       A + 3 * o, S + o, NULL, NULL, F, ro);
            if ((t + 1) % sample_every == 0) {
                if (samples) stress_chain(n, ns, R + 3 * o, A + 3 * o, S + o, samples + 12 * ((int64_t)n_chains * q + k));
                ++q;
            }
        }
        free(F);
        free(ro);
    }
    return n_samples;
}

/* ---- Multiple-tau correlator, by its definition --------------------------
 * Level 0 is the sample series itself; level l >= 1 is the series of
 * pairwise means of consecutive, non-overlapping pairs of level l-1.  At
 * every level, C[l][k] = sum_{n >= k} x_l[n] * y_l[n-k] and
 * cnt[l][k] = max(0, len_l - k).  Lag k at level l stands for
 * tau = k * 2^l sampling intervals.  x and y: [T] series of one quantity. */
void ssp_oracle_multitau(int64_t T, const double* x, const double* y, int levels, int lags, double* C,
                         int64_t* cnt)
{
    double* xl = (double*)malloc(sizeof(double) * (size_t)(T > 0 ? T : 1));
    double* yl = (double*)malloc(sizeof(double) * (size_t)(T > 0 ? T : 1));
    int64_t len = T;
    for (int64_t n = 0; n < T; ++n) {
        xl[n] = x[n];
        yl[n] = y[n];
    }
    for (int l = 0; l < levels; ++l) {
        if (l > 0) {
            int64_t half = len / 2;
            for (int64_t n = 0; n < half; ++n) {
                xl[n] = (xl[2 * n] + xl[2 * n + 1]) * 0.5;
                yl[n] = (yl[2 * n] + yl[2 * n + 1]) * 0.5;
            }
            len = half;
        }
        for (int k = 0; k < lags; ++k) {
            double acc = 0.0;
            for (int64_t n = k; n < len; ++n) acc += xl[n] * yl[n - k];
            C[(int64_t)l * lags + k] = acc;
            cnt[(int64_t)l * lags + k] = len > k ? len - k : 0;
        }
    }
    free(xl);
    free(yl);
}

/* ---- Frozen-event step and discrete adjoint ------------------------------
 * The derivative of a finite-time stress with respect to the flow rate or the
 * slip-spring strength is taken conditioned on the recorded hop, creation and
 * destruction events and on the random normals (pathwise derivative of the
 * Euler map of Sec. 3.1 with the events held fixed).  The dependence of the
 * event probabilities on the parameters is not part of it. */

/* One step whose slot decisions are given: the substep-1 move with the
 * current slots, then S := S_next; a slot that goes from empty to occupied is
 * a spring created at bead S_next with anchor R' + sqrt(N_s/3) g (the anchor
 * normals of that slot and step); a slot that goes from occupied to empty is a
 * destroyed spring. */
void ssp_oracle_step_forced(int n_chains, const int32_t* N, const int64_t* off, const int64_t* chain_id,
                            const double* kappa, double dt, double ns, uint64_t seed, int64_t step, double* R,
                            double* A, int32_t* S, const int32_t* S_next)
{
    const double anchor_sd = sqrt(ns / 3.0);
#pragma omp parallel for schedule(dynamic, 8)
    for (int k = 0; k < n_chains; ++k) {
        int n = N[k];
        int64_t o = off[k];
        double* r = R + 3 * o;
        double* a = A + 3 * o;
        int32_t* s = S + o;
        const int32_t* sn = S_next + o;
        double* F = (double*)malloc(sizeof(double) * 3 * (size_t)n);
        double* ro = (double*)malloc(sizeof(double) * 3 * (size_t)n);
        move_chain(n, chain_id[k], kappa + 9 * (int64_t)k, dt, ns, seed, step, r, a, s, F, ro);
        for (int j = 0; j < n; ++j) {
            if (s[j] < 0 && sn[j] >= 0) {
                double g[3];
                ssp_oracle_normals3(seed, P_ANCHOR, j, chain_id[k], step, g);
                for (int d = 0; d < 3; ++d) a[3 * j + d] = r[3 * sn[j] + d] + anchor_sd * g[d];
            } else if (sn[j] < 0) {
                a[3 * j] = a[3 * j + 1] = a[3 * j + 2] = 0.0;
            }
            s[j] = sn[j];
        }
        free(F);
        free(ro);
    }
}

/* Indices of the stress components: xx yy zz xy yz zx. */
static const int COMP_A[6] = {0, 1, 2, 0, 1, 2};
static const int COMP_B[6] = {0, 1, 2, 1, 2, 0};

/* Gradient of J = sigma_comp(R_T) of every chain with respect to the velocity
 * gradient kappa (9 entries, constant over the window) and to N_s, by the
 * reverse recursion through steps T-1 .. 0 of the window.
 *
 * Rt [(T+1)][tot][3], At [(T+1)][tot][3], St [(T+1)][tot]: the state before
 * step step0 + n at index n (n = 0..T).  kappa [M][9].  If init_window, the
 * anchors at index 0 are the sampled equilibrium anchors A = R_S +
 * sqrt(N_s/3) g(INIT_ANCHOR) and their N_s dependence is included.
 * Outputs gk [M][9], gns [M].
 *
 * Per step n (state x_n = (R_n, A_n), slots S_n -> S_{n+1}):
 *   R_{n+1} = R_n + dt (F(R_n, A_n; S_n) + kappa R_n) + noise,
 *   A_{n+1,j} = A_{n,j} + dt kappa A_{n,j}        (slot occupied before and after),
 *   A_{n+1,j} = R_{n+1,S_{n+1,j}} + sqrt(N_s/3) g  (slot created in step n);
 * with lR = dJ/dR_{n+1}, lA = dJ/dA_{n+1}:
 *   lR[e_j] += lA[j] for created slots, dJ/dN_s += lA[j] . g / (2 sqrt(3 N_s));
 *   dJ/dR_n = lR + dt (L lR - (3/N_s) c lR + kappa^T lR)   (L: bond Laplacian,
 *             c_i: springs on bead i at step n);
 *   dJ/dA_n[j] = (1 + dt kappa^T) lA[j] (surviving) + dt (3/N_s) lR[S_{n,j}];
 *   dJ/dkappa_ab += dt (sum_i lR_ia R_{n,i,b} + sum_surviving j lA_ja A_{n,j,b});
 *   dJ/dN_s += dt (3/N_s^2) sum_j lR[S_{n,j}] . (R_{n,S_j} - A_{n,j}). */
void ssp_oracle_adjoint(int n_chains, const int32_t* N, const int64_t* off, const int64_t* chain_id,
                        const double* kappa, double dt, double ns, uint64_t seed, int64_t step0, int64_t T,
                        const double* Rt, const double* At, const int32_t* St, int64_t tot, int comp,
                        int init_window, double* gk, double* gns)
{
    const double ks = 3.0 / ns;
    const double dsig = 1.0 / (2.0 * sqrt(3.0 * ns));
    const int ca = COMP_A[comp], cb = COMP_B[comp];
#pragma omp parallel for schedule(dynamic, 4)
    for (int k = 0; k < n_chains; ++k) {
        const int n = N[k];
        const int64_t o = off[k];
        const double* kap = kappa + 9 * (int64_t)k;
        double* lR = (double*)calloc(3 * (size_t)n, sizeof(double));
        double* lA = (double*)calloc(3 * (size_t)n, sizeof(double));
        double* nR = (double*)calloc(3 * (size_t)n, sizeof(double));
        double* nA = (double*)calloc(3 * (size_t)n, sizeof(double));
        int* cnt = (int*)calloc((size_t)n, sizeof(int));
        double G[9] = {0}, Gns = 0.0;
        /* seed: dJ/dR_T of sigma_ab = sum_i 3 b_ia b_ib */
        const double* RT = Rt + 3 * (T * tot + o);
        for (int i = 0; i + 1 < n; ++i) {
            double b[3];
            for (int d = 0; d < 3; ++d) b[d] = RT[3 * (i + 1) + d] - RT[3 * i + d];
            double g[3] = {0.0, 0.0, 0.0};
            g[ca] += 3.0 * b[cb];
            g[cb] += 3.0 * b[ca];
            for (int d = 0; d < 3; ++d) {
                lR[3 * (i + 1) + d] += g[d];
                lR[3 * i + d] -= g[d];
            }
        }
        for (int64_t m = T - 1; m >= 0; --m) {
            const double* Rn = Rt + 3 * (m * tot + o);
            const double* An = At + 3 * (m * tot + o);
            const int32_t* Sn = St + m * tot + o;
            const int32_t* S1 = St + (m + 1) * tot + o;
            /* created slots feed their anchor adjoint to the end bead */
            for (int j = 0; j < n; ++j) {
                if (Sn[j] < 0 && S1[j] >= 0) {
                    double g[3];
                    ssp_oracle_normals3(seed, P_ANCHOR, j, chain_id[k], step0 + m, g);
                    for (int d = 0; d < 3; ++d) {
                        lR[3 * S1[j] + d] += lA[3 * j + d];
                        Gns += lA[3 * j + d] * g[d] * dsig;
                    }
                }
            }
            for (int i = 0; i < n; ++i) cnt[i] = 0;
            for (int j = 0; j < n; ++j)
                if (Sn[j] >= 0) ++cnt[Sn[j]];
            /* parameter terms of step m (use lR = dJ/dR_{m+1}, lA = dJ/dA_{m+1}) */
            for (int i = 0; i < n; ++i)
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) G[3 * a + b] += dt * lR[3 * i + a] * Rn[3 * i + b];
            for (int j = 0; j < n; ++j) {
                if (Sn[j] >= 0 && S1[j] >= 0)
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) G[3 * a + b] += dt * lA[3 * j + a] * An[3 * j + b];
                if (Sn[j] >= 0) {
                    const int i = Sn[j];
                    for (int d = 0; d < 3; ++d) Gns += dt * (3.0 / (ns * ns)) * lR[3 * i + d] * (Rn[3 * i + d] - An[3 * j + d]);
                }
            }
            /* dJ/dR_m */
            for (int i = 0; i < n; ++i) {
                for (int d = 0; d < 3; ++d) {
                    double lap = 0.0;
                    if (i + 1 < n) lap += 3.0 * (lR[3 * (i + 1) + d] - lR[3 * i + d]);
                    if (i > 0) lap -= 3.0 * (lR[3 * i + d] - lR[3 * (i - 1) + d]);
                    double kt = kap[0 * 3 + d] * lR[3 * i + 0] + kap[1 * 3 + d] * lR[3 * i + 1] + kap[2 * 3 + d] * lR[3 * i + 2];
                    nR[3 * i + d] = lR[3 * i + d] + dt * (lap - ks * cnt[i] * lR[3 * i + d] + kt);
                }
            }
            /* dJ/dA_m */
            for (int j = 0; j < n; ++j) {
                for (int d = 0; d < 3; ++d) nA[3 * j + d] = 0.0;
                if (Sn[j] < 0) continue;
                if (S1[j] >= 0) {
                    for (int d = 0; d < 3; ++d) {
                        double kt = kap[0 * 3 + d] * lA[3 * j + 0] + kap[1 * 3 + d] * lA[3 * j + 1] + kap[2 * 3 + d] * lA[3 * j + 2];
                        nA[3 * j + d] = lA[3 * j + d] + dt * kt;
                    }
                }
                for (int d = 0; d < 3; ++d) nA[3 * j + d] += dt * ks * lR[3 * Sn[j] + d];
            }
            for (int q = 0; q < 3 * n; ++q) {
                lR[q] = nR[q];
                lA[q] = nA[q];
            }
        }
        if (init_window) {
            const int32_t* S0 = St + o;
            for (int j = 0; j < n; ++j) {
                if (S0[j] < 0) continue;
                double g[3];
                ssp_oracle_normals3(seed, P_INIT_ANCHOR, j, chain_id[k], 0, g);
                for (int d = 0; d < 3; ++d) Gns += lA[3 * j + d] * g[d] * dsig;
            }
        }
        for (int q = 0; q < 9; ++q) gk[9 * (int64_t)k + q] = G[q];
        gns[k] = Gns;
        free(lR);
        free(lA);
        free(nR);
        free(nA);
        free(cnt);
    }
}
