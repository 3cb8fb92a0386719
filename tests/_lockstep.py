"""Lock-step comparison of the GPU path with the FP64 oracle, step by step,
for chains of any lengths (helpers for the GPU parity tests).

Per step (Sec. 3.1 step map), both sides advance the same chains (same seed,
same global chain ids, same velocity gradients) and every translation-
invariant quantity is compared: bond vectors R_{i+1} - R_i and anchor offsets
d_j = R_{S_j} - A_j to the per-step bar, relative to max(|oracle|, 0.58)
(0.58 = rms bond component), and every slot's bead index S_j exactly.

A decision may differ only where the oracle's margin |u - P| is below 1e-5
(a tie: an FP32 probability carries ~1e-7 relative error).  Then the tie is
counted and the oracle adopts the GPU's decision for that step (teacher
forcing: the step is re-run from the saved state with the GPU's slot row, by
the oracle's frozen-event step), so that every chain stays compared to the
end.  On the FP64 path no tie is tolerated.

Bonds and anchor offsets next to strongly stretched bonds (elongation beyond
the Rouse instability stretches bonds to hundreds of times their rest length)
carry an extra, derived allowance on the FP32 path.  A bead there sits where
bond tensions of size k_b |b| balance, so any relative perturbation eps of
those forces moves it by eps k_b |b| / k, k the stiffness that restores the
compared quantity: k_b for a bond (k_b / k = 1), the slip spring's
k_s = 3/N_s for an anchor offset (k_b / k = N_s).  binary32 arithmetic
perturbs the forces by a few units of 2^-24 per step (the rounded normals,
bond vectors, stiffness constants and sums), so the allowance is
8 * 2^-24 * (k_b / k) * |b|, |b| the longest bond at the compared bond's or
spring's beads (oracle): below 1e-7 near rest length, about 2e-4 at
|b| = 500.  (On the CPU the oracle's own FP64 step with only its normals
rounded to binary32 moves such an anchor offset by about 5e-9 |b|.)
"""
from __future__ import annotations

import numpy as np

SCALE = 0.58
TIE = 1e-5
STRETCH = 8.0 * 2.0 ** -24  # binary32 force perturbation per step, in units of the bond tension


class Layout:
    """Index tables for chains of lengths N packed back to back."""

    def __init__(self, N):
        self.N = np.asarray(N, dtype=np.int64)
        self.off = np.zeros(len(self.N), dtype=np.int64)
        if len(self.N) > 1:
            self.off[1:] = np.cumsum(self.N[:-1])
        self.total = int(self.N.sum())
        self.chain = np.repeat(np.arange(len(self.N)), self.N)
        last = self.off + self.N - 1
        self.has_bond = np.ones(self.total, dtype=bool)
        self.has_bond[last] = False
        self.bond_idx = np.nonzero(self.has_bond)[0]

    def bond_lengths(self, R):
        """Per bond (bead i -> i+1): the longest of it and its neighbouring bonds."""
        b = np.linalg.norm(R[self.bond_idx + 1] - R[self.bond_idx], axis=1)
        per_bead = np.zeros(self.total)
        per_bead[self.bond_idx] = b
        left = np.zeros(self.total)
        left[self.bond_idx + 1] = b
        right_next = np.zeros(self.total)
        right_next[:-1] = per_bead[1:]
        # neighbours of bond i: bond i-1 (left of bead i) and bond i+1 (right of bead i+1);
        # a chain's first/last bond has zeros there (no bond crosses chains)
        nxt = np.where(self.has_bond[self.bond_idx + 1], right_next[self.bond_idx], 0.0)
        return np.maximum(np.maximum(b, left[self.bond_idx]), nxt)

    def adjacent_bond(self, R, S):
        """Per slot: the length of the longer bond at the slot's bead (0 if empty)."""
        b = np.linalg.norm(R[self.bond_idx + 1] - R[self.bond_idx], axis=1)
        bl = np.zeros(self.total)
        bl[self.bond_idx] = b              # bond to the right of a bead
        br = np.zeros(self.total)
        br[self.bond_idx + 1] = b          # bond to the left of a bead
        both = np.maximum(bl, br)
        occ = S >= 0
        bead = self.off[self.chain] + np.where(occ, S, 0)
        return np.where(occ, both[bead], 0.0)

    def invariants(self, R, A, S):
        """bonds [n_bonds][3] (bead i -> i+1 of each chain), anchor offsets
        [total][3] (0 where empty), occupancy mask."""
        b = R[self.bond_idx + 1] - R[self.bond_idx]
        occ = S >= 0
        bead = self.off[self.chain] + np.where(occ, S, 0)
        d = np.where(occ[:, None], R[bead] - A, 0.0)
        return b, d, occ


def rel_err(g, o):
    return np.abs(g - o) / np.maximum(np.abs(o), SCALE)


def _worst_report(lay, o, R, A, S, bg, bo, dg, do, occ):
    """Where the largest error sits: chain (global id), bead or slot, values."""
    out = []
    eb = rel_err(bg, bo)
    i, c = np.unravel_index(np.argmax(eb), eb.shape)
    bead = lay.bond_idx[i]
    k = lay.chain[bead]
    out.append(f"bond: chain {o.chain_ids[k]} (N = {lay.N[k]}) bead {bead - lay.off[k]} comp {c}: "
               f"gpu {bg[i, c]:.9g} oracle {bo[i, c]:.9g}; |R| there {np.abs(o.R[bead]).max():.4g}")
    if occ.any():
        ed = np.where(occ[:, None], rel_err(dg, do), 0.0)
        j, c = np.unravel_index(np.argmax(ed), ed.shape)
        k = lay.chain[j]
        sb = lay.off[k] + o.S[j]
        out.append(f"anchor offset: chain {o.chain_ids[k]} (N = {lay.N[k]}) slot {j - lay.off[k]} at bead {o.S[j]} "
                   f"comp {c}: gpu {dg[j, c]:.9g} oracle {do[j, c]:.9g}; |R_S| {np.abs(o.R[sb]).max():.4g}, "
                   f"|A| {np.abs(o.A[j]).max():.4g}, chain extent {np.ptp(o.R[lay.off[k]:lay.off[k] + lay.N[k]], axis=0)}")
    return "; ".join(out)


def lockstep(e, o, steps, kappa_elem=None, kappa_chain=None, tol=1e-5, fp64=False, on_step=None,
             resync_every=None):
    """Advance GPU ensemble `e` and oracle ensemble `o` (the same chains in the
    same order) by `steps` steps, comparing after every step.

    resync_every: for runs longer than the 1e3 steps over which the per-step
    bar applies, the oracle restarts from the GPU's state (its FP64 view,
    hi + lo exactly) at every multiple of this many steps, so that each window
    is compared from a common state; without it the run is compared
    free-running from the common initial state.

    kappa_elem: [E][9] for the GPU (None: at rest); kappa_chain: [M][9] for
    the oracle.  on_step(t, o, events, pre): called after each compared step
    with the oracle's event bits of that step and its state (R, A, S) before it.
    Returns dict(worst, ties, tie_margins, steps)."""
    lay = Layout(o.N)
    worst = 0.0
    ties = 0
    tie_margins = []
    window_worst = []
    for t in range(steps):
        if resync_every and t > 0 and t % resync_every == 0:
            window_worst.append(worst)
            worst = 0.0
            o.R[:], o.A[:], o.S[:] = R, np.where((S >= 0)[:, None], A, 0.0), S
        saved = (o.R.copy(), o.A.copy(), o.S.copy(), o.step_index)
        e.step(1, kappa_elem)
        events, margin = o.step(kappa_chain, want_events=True)
        R, A, S = (x.cpu().numpy() for x in e.state())
        mism = S != o.S
        if mism.any():
            slots = np.nonzero(mism)[0]
            m = margin[slots]
            assert not fp64, f"decision mismatch on the FP64 path at step {t}: slots {slots}"
            assert np.all(m < TIE), f"decision mismatch outside a tie at step {t}: slots {slots}, margins {m}"
            ties += len(np.unique(lay.chain[slots]))
            tie_margins.extend(m.tolist())
            # teacher forcing: redo the oracle's step with the GPU's slot row
            o.R[:], o.A[:], o.S[:] = saved[0], saved[1], saved[2]
            o.step_index = saved[3]
            o.step_forced(S, kappa_chain)
            assert np.array_equal(S, o.S)
        bg, dg, _ = lay.invariants(R, A, S)
        bo, do, occ = lay.invariants(o.R, o.A, o.S)
        eb = 0.0
        if len(bg):
            allow_b = 0.0 if fp64 else STRETCH * lay.bond_lengths(o.R)[:, None]
            eb = (np.abs(bg - bo) / (np.maximum(np.abs(bo), SCALE) + allow_b / tol)).max()
        ed = 0.0
        if occ.any():
            # the offset bar in units of tol: tol max(|d|, 0.58) plus the
            # stretched-bond allowance (FP32 only; see the module docstring)
            allow = 0.0 if fp64 else STRETCH * o.ns * lay.adjacent_bond(o.R, o.S)[occ][:, None]
            ed = (np.abs(dg[occ] - do[occ]) / (np.maximum(np.abs(do[occ]), SCALE) + allow / tol)).max()
        worst = max(worst, eb, ed)
        if not (eb <= tol and ed <= tol):
            raise AssertionError(f"step {t}: bond error {eb:.3e}, anchor-offset error {ed:.3e} (bar {tol}); "
                                 + _worst_report(lay, o, R, A, S, bg, bo, dg, do, occ))
        if on_step is not None:
            on_step(t, o, events, saved)
    window_worst.append(worst)
    return {"worst": max(window_worst), "window_worst": window_worst, "ties": ties, "tie_margins": tie_margins,
            "steps": steps}
