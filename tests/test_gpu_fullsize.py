"""Parity at the full workload sizes and lengths, in the launch configuration
the benchmark uses, checked on sampled chains the oracle computes (a chain's
trajectory depends only on the seed, its global chain id and the step).

For each workload:
  1. the full-size ensemble runs the workload's whole length on the GPU;
  2. a small GPU ensemble of the sampled chains (same global ids, seeds and
     velocity gradients) runs the same steps one at a time in lock step with
     the FP64 oracle: every step's bonds and anchor offsets within the per-step
     bar (1e-5 relative to max(|x|, 0.58) on the FP32 path), every decision
     identical except margin-checked ties (|u - P| < 1e-5), where the oracle
     adopts the GPU's decision (teacher forcing, so every chain stays compared);
  3. the small ensemble's final state equals the full-size run's state of the
     same chains bit for bit (trajectories do not depend on the launch layout),
     so the lock-step comparison covers the full-size run.

The per-step bar holds over 1e3 steps.  Beyond that an FP32 trajectory under
strong flow leaves the FP64 one, because the flow amplifies small deviations
(a deviation dy of a bead grows into gamma_dot t dy in x under shear; under
elongation it grows with the stretch) while the chain and its springs relax
them only on the chain's own relaxation times.  Runs longer than 1e3 steps
under flow are therefore compared in windows of 1e3 steps: at each window
start the oracle restarts from the GPU's state, and within the window every
step meets the per-step bar.  The runs at rest are compared free-running.
"""
import math

import numpy as np
import pytest

import oracle
from paper_1106_2899_amd import workloads

from _lockstep import Layout, lockstep

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _bitwise_same_chains(big, small, ids):
    """The small ensemble (chains `ids` of `big`, in order) holds exactly the
    big ensemble's state of those chains."""
    Rb, Ab, Sb = (x.cpu().numpy() for x in big.state())
    Rs, As, Ss = (x.cpu().numpy() for x in small.state())
    for q, k in enumerate(ids):
        n = int(big.N[k])
        sb = slice(int(big.offsets[k]), int(big.offsets[k]) + n)
        ss = slice(int(small.offsets[q]), int(small.offsets[q]) + n)
        assert np.array_equal(Sb[sb], Ss[ss]), k
        assert np.array_equal(Rb[sb], Rs[ss]), k
        occ = Sb[sb] >= 0
        assert np.array_equal(Ab[sb][occ], As[ss][occ]), k


def _sampled_lockstep(big, ids, steps, kap_elem_of_chain, seed, sample_every, elem_groups=None, on_step=None,
                      resync_every=None):
    """Runs the chains `ids` as a small ensemble in lock step with the oracle
    for `steps` steps from the same initial state; returns (small, oracle, stats)."""
    from paper_1106_2899_amd.ensemble import Ensemble
    N = [int(big.N[i]) for i in ids]
    kchain = np.ascontiguousarray(kap_elem_of_chain[ids])
    if elem_groups is None:
        E, offs = len(ids), np.arange(len(ids) + 1)
    else:
        E, offs = len(elem_groups) - 1, np.asarray(elem_groups)
    small = Ensemble(N, n_elements=E, element_offsets=offs, chain_ids=np.asarray(ids, dtype=np.int64),
                     precision="fp32", seed=seed, sample_every=sample_every, corr_levels=0,
                     series_capacity=(steps // sample_every if elem_groups is not None else 0)).init()
    kap_small = torch.as_tensor(kchain[offs[:-1]], dtype=torch.float64, device="cuda")
    o = oracle.Ensemble(N, chain_ids=ids, seed=seed).init()
    stats = lockstep(small, o, steps, kappa_elem=kap_small, kappa_chain=kchain, on_step=on_step,
                     resync_every=resync_every)
    return small, o, stats


def test_lve_16384x32_bench_launch_sampled_chains():
    """The benchmark's 5000-step graph launch of 16384 x N = 32 (correlator on)."""
    _need_gpu()
    from paper_1106_2899_amd.ensemble import Ensemble
    w = workloads.linear_viscoelasticity()
    steps = 5000
    e = Ensemble(w.n_beads, precision="fp32", seed=w.seed, sample_every=w.sample_every, corr_levels=16,
                 corr_batches=16, max_steps_per_launch=steps, use_graph=True).init()
    e.step(steps)
    ids = np.linspace(0, w.n_chains - 1, 48).astype(np.int64)
    kchain = np.zeros((w.n_chains, 9))
    small, _, st = _sampled_lockstep(e, ids, steps, kchain, w.seed, w.sample_every)
    print(f"lve 48 sampled chains x {steps} steps: worst {st['worst']:.2e}, ties {st['ties']}")
    _bitwise_same_chains(e, small, ids)
    G = e.correlator()
    assert G["counts"][0, 0] == steps // w.sample_every and np.isfinite(G["G"]).all()


def _series_bar(sum_b2, nbonds, tol=1e-5):
    """Bound on |gpu - oracle| of an element's summed off-diagonal stress
    sigma_ab = sum 3 b_a b_b implied by the per-step bar on every bond
    component, |db_c| <= tol (|b_c| + 0.58): per bond
    |d(3 b_a b_b)| <= 3 tol (2 |b_a| |b_b| + 0.58 (|b_a| + |b_b|))
                   <= 3 tol (|b|^2 + 0.82 |b|) <= tol (4.25 |b|^2 + 1.25),
    summed over the element's bonds; sum |b|^2 = (tr sum sigma + 3 sum N) / 3."""
    return tol * (4.25 * sum_b2 + 1.25 * nbonds)


def test_startup_shear_full_length_sampled_chains_and_element_series():
    """1,048,576 chains (4096 elements x 256, N = 32), each element its own
    shear rate, 2e4 steps replayed as one captured graph; a whole element and
    40 chains across the ensemble in lock step; the element's viscosity-growth
    series against the oracle's (teacher-forced) sums."""
    _need_gpu()
    from paper_1106_2899_amd.ensemble import Ensemble
    w = workloads.startup_shear()
    steps = w.steps
    T = steps // w.sample_every
    e = Ensemble(w.n_beads, n_elements=w.n_elements, element_offsets=w.element_offsets, precision="fp32",
                 seed=w.seed, sample_every=w.sample_every, corr_levels=0, series_capacity=T, use_graph=True).init()
    kap = torch.as_tensor(w.kappa.reshape(w.n_elements, 9), dtype=torch.float64, device="cuda")
    e.step(steps, kap)  # one graph launch
    ser = e.element_series().cpu().numpy()
    assert ser.shape == (w.n_elements, T, 6)
    kchain = np.repeat(w.kappa.reshape(w.n_elements, 9), np.diff(w.element_offsets), axis=0)
    el = int(np.argmax(w.rates))  # the fastest element: the most stretched chains
    lo, hi = int(w.element_offsets[el]), int(w.element_offsets[el + 1])
    spread = np.linspace(0, w.n_chains - 1, 40).astype(np.int64)
    spread = spread[(spread < lo) | (spread >= hi)]
    ids = np.concatenate([np.arange(lo, hi, dtype=np.int64), spread])
    groups = [0] + list(range(hi - lo, len(ids) + 1))  # the element, then one element per spread chain
    want = np.zeros((T, 6))
    nb = hi - lo

    def on_step(t, o, ev, pre):
        if (t + 1) % w.sample_every == 0:
            want[(t + 1) // w.sample_every - 1] = o.stress()[:nb, :6].sum(axis=0)

    small, o, st = _sampled_lockstep(e, ids, steps, kchain, w.seed, w.sample_every, elem_groups=groups,
                                     on_step=on_step, resync_every=1000)
    print(f"startup shear: element {el} (rate {w.rates[el]:.3g}) + {len(spread)} chains x {steps} steps: "
          f"worst {st['worst']:.2e}, ties {st['ties']}; per window {np.round(st['window_worst'], 8)}")
    _bitwise_same_chains(e, small, ids)
    got_small = small.element_series().cpu().numpy()[0]
    np.testing.assert_allclose(got_small, ser[el], rtol=1e-12, atol=1e-12 * np.abs(ser[el]).max())
    tr = want[:, 0] + want[:, 1] + want[:, 2] + 3 * 32 * nb
    bar = _series_bar(tr / 3.0, 31 * nb)
    for c in (3, 4, 5):
        dev = np.abs(ser[el][:, c] - want[:, c])
        assert np.all(dev <= bar), (c, (dev / bar).max())
    print("element series: max |gpu - oracle| / bar =", max((np.abs(ser[el][:, c] - want[:, c]) / bar).max()
                                                          for c in (3, 4, 5)))


def test_polydisperse_full_length_sampled_chains():
    """2^18 chains, N uniform in 16..128, shear and uniaxial elements, 1e4
    steps (rate x time <= 10); sampled chains include the longest chains of
    the fastest uniaxial elements (the stretched, large-coordinate regime)."""
    _need_gpu()
    from paper_1106_2899_amd.ensemble import Ensemble
    w = workloads.polydisperse()
    steps = w.steps
    e = Ensemble(w.n_beads, n_elements=w.n_elements, element_offsets=w.element_offsets, precision="fp32",
                 seed=w.seed, sample_every=w.sample_every, corr_levels=0, use_graph=True).init()
    kap = torch.as_tensor(w.kappa.reshape(w.n_elements, 9), dtype=torch.float64, device="cuda")
    e.step(steps, kap)
    kchain = np.repeat(w.kappa.reshape(w.n_elements, 9), np.diff(w.element_offsets), axis=0)
    uni = np.nonzero(w.kinds == 1)[0]
    fast = uni[np.argsort(w.rates[uni])[-4:]]
    stretched = []
    for el in fast:
        lo, hi = int(w.element_offsets[el]), int(w.element_offsets[el + 1])
        stretched += list(lo + np.argsort(w.n_beads[lo:hi])[-2:])
    spread = list(np.linspace(0, w.n_chains - 1, 32).astype(np.int64))
    ids = np.array(sorted(set(int(i) for i in stretched + spread)), dtype=np.int64)
    small, _, st = _sampled_lockstep(e, ids, steps, kchain, w.seed, w.sample_every, resync_every=1000)
    print(f"polydisperse: {len(ids)} chains (incl. N = {sorted(int(w.n_beads[i]) for i in stretched)} at "
          f"elongation rates {np.round(w.rates[fast], 4)}) x {steps} steps: worst {st['worst']:.2e}, ties {st['ties']}; "
          f"per window {np.round(st['window_worst'], 8)}")
    _bitwise_same_chains(e, small, ids)


ADJ_IDS = np.array([0, 7777, 13000, 29999, 40000, 52000, 60001, 65535], dtype=np.int64)


@pytest.mark.parametrize("stored", [False, True], ids=["checkpointed", "stored_400"])
def test_differentiation_full_size_sampled_chains(stored):
    """All 65536 chains of N = 64 at shear rate 0.01; the checkpointed window
    at its full length (2000 steps, a checkpoint every 100), and a 400-step
    window recorded as one stored segment (about 22 GB; the full 2000-step
    one, 110 GB, is timed by the benchmark).  Per-chain gradients of the final
    sigma_xy against the FP64 oracle's adjoint of the same events."""
    _need_gpu()
    from paper_1106_2899_amd.ensemble import Ensemble
    w = workloads.differentiation()
    steps, ckpt = (400, 400) if stored else (w.steps, w.extra["checkpoint_every"])
    e = Ensemble(w.n_beads, precision="fp32", seed=w.seed, sample_every=10, corr_levels=0).init()
    kap = w.kappa.reshape(1, 9)
    e.forward_record(steps, ckpt, kap)
    g = e.adjoint(component=3).cpu().numpy()
    ids = ADJ_IDS
    o = oracle.Ensemble([int(w.n_beads[i]) for i in ids], chain_ids=ids, seed=w.seed).init()
    Rt, At, St = o.run_record(steps, kap)
    gk, gns = o.adjoint(Rt, At, St, kap, comp=3)
    R, A, S = (x.cpu().numpy() for x in e.state())
    offsets = e.offsets
    e.close()
    compared = 0
    worst_k = worst_n = 0.0
    # relative to max(|oracle|, rms over the sampled chains), as the per-step
    # metric is relative to max(|x|, rms bond): a chain's gradient can cross
    # zero, where a purely relative error means nothing
    sk = np.sqrt(np.mean(gk[:, 0, 1] ** 2))
    sn = np.sqrt(np.mean(gns ** 2))
    for q, k in enumerate(ids):
        sl = slice(int(offsets[k]), int(offsets[k]) + 64)
        if not np.array_equal(S[sl], o.S[o.off[q]:o.off[q] + 64]):
            continue  # a tie changed an event of this chain (R15): its gradient is another path's
        compared += 1
        worst_k = max(worst_k, abs(g[k, 1] - gk[q, 0, 1]) / max(abs(gk[q, 0, 1]), sk))
        worst_n = max(worst_n, abs(g[k, 9] - gns[q]) / max(abs(gns[q]), sn))
        print(f"  chain {k}: d/dkappa_xy gpu {g[k, 1]:.9g} oracle {gk[q, 0, 1]:.9g}; "
              f"d/dN_s gpu {g[k, 9]:.9g} oracle {gns[q]:.9g}")
    print(f"adjoint ({'stored' if stored else 'checkpointed'}): {compared}/{len(ids)} chains compared, "
          f"max rel err d/dkappa_xy {worst_k:.2e}, d/dN_s {worst_n:.2e}")
    assert compared >= len(ids) - 1, compared
    assert worst_k <= 1e-4 and worst_n <= 1e-4, (worst_k, worst_n)
