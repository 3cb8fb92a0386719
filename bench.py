"""Benchmark of the slip-spring ensemble step on one MI355X.

Headline workload: the equilibrium linear-viscoelasticity ensemble, 16384
chains of N = 32 beads (N_0 = 4, N_s = 0.5, zeta_s = 0.1, dt = 0.01), FP32 bead
dynamics with FP64 stress, stress sampled every 10 steps into the FP64
multiple-tau correlator (16 levels x 16 lags).  One benchmark step is one
ssp_step call of 5000 time steps over the whole ensemble (every row of the hot
path: RNG, forces, Euler move, hops, reconstruction, stress, correlator),
replayed from a captured hipGraph; the default 20 steps are the full 1e5-step
run.  Inputs are resident in HBM before the timed region.

Printed: one JSON line with bead-steps/s of the batched FP32 path; the plain
FP64 path at the same shape and on the 64 x N = 8 equilibrium workload; the
VALU roofline of the step kernel (launch durations from HIP events on the
launch stream); the adjoint/forward time ratio (a checkpoint every 100 steps,
and the window stored as one segment); the start-up shear (4096 elements x 256
chains, 2e4 steps) and polydisperse (2^18 chains, 1e4 steps) workloads at full
length, each with its own roofline fraction; the shapes of the paper's
timing table (context, beside the paper's GPU seconds); and, from the CPU
leg, the FP64 oracle timed on the host cores (all threads and one thread,
with the CPU model) and the accuracy of every number against that oracle:
the per-step error and ties of sampled chains in lock step, G(t) of the
headline run in units of its standard error, the final state of the FP64
run, and the adjoint's per-chain gradients.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

CHAINS, BEADS, SAMPLE_EVERY = 16384, 32, 10
MD_STEPS_PER_BENCH_STEP = 5000  # 20 bench steps = the whole 1e5-step run
PEAK_LANE_SLOTS = 256 * 4 * 16 * 2.4e9  # CUs x SIMDs x lanes x clock: full-rate VALU lane-issue slots/s
QUEUE_KERNEL = "k_step_queue<float,32,1,false,false>"
# The shapes of the paper's timing table (Sec. 4): N x M with N M = 65536
# beads, 1e4 steps from equilibrium, at rest and under simple shear at rate
# 0.05, with the seconds the paper's GPU (FP32, 2009) took for each.
PAPER_TABLE_SHAPES = [(16, 4096, 0.0, 0.897), (16, 4096, 0.05, 0.895), (32, 2048, 0.0, 0.902),
                      (32, 2048, 0.05, 0.895), (64, 1024, 0.0, 0.870), (64, 1024, 0.05, 0.863),
                      (128, 512, 0.0, 0.845), (128, 512, 0.05, 0.840)]
PAPER_TABLE_STEPS = 10_000


def _log(msg):
    """Stage progress on stderr (stdout carries only the JSON line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def algorithmic_valu_slots(sample_every: int = SAMPLE_EVERY, n0: float = 4.0, flow_entries: float = 0.0) -> float:
    """VALU issue slots per bead-step that the method needs on this workload.
    A slot is one wave64 instruction issued over 4 SIMD cycles (16 lanes per
    cycle), so the chip's peak is 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
    lane-slots/s.  Each operation is weighted by its issue cost measured on
    gfx950 with the probe library (SIMD cycles per wave64 instruction / 4):
    0.5 for FP32 add/sub/mul/FMA, 32-bit integer add/sub, and/or/xor, the
    three-input bitop, v_mov and right shifts; 1 for the 32x32->64 integer
    multiply-add, compares, selects, min/max, alignbit, conversions, DPP
    moves and FP64 add/mul/FMA; 2 for the FP32 transcendentals log, exp,
    sqrt, sin, cos and rcp.  The arithmetic is the path's (compensated FP32
    positions, FP64 stress) with the random stream at its minimum of five
    words per bead-step:
      random words: 1.5 Box-Muller pairs (3 words) + hop + reconstruction
        = 1.25 Philox4x32-10 blocks x 10 rounds x (2 multiply-adds
        + 2 three-input xors)                                           ->  37.5
      Box-Muller, 1.5 pairs x (2 uniforms x (alignbit + add) 3, log 2,
        mul 0.5, sqrt 2, sin 2, cos 2, 2 mul 1)                         ->  18.75
      bonds from compensated positions, 3 x (2 sub + add)               ->   4.5
      move: bond-force difference 1.5, two FMAs per component 3,
        compensated position update 12 x 0.5                            ->  10.5
      spring-force gather, 3 adds per spring                            ->   1.5 / N_0
      hop per occupied slot: post-move offset 1.5, two energy
        differences 2 x 3, two probabilities 2 x (mul, exp, add, rcp,
        mul, min) 13, decision 3.5                                      ->  24 / N_0
      reconstruction word test (one compare)                            ->   1
      anchor offsets for the next step (compensated), per spring       ->   4.5 / N_0
      stress and virtual stress (FP64), per sample: per bead 3 cvt
        + 6 FMA, per spring the same                                    ->  (9 + 9 / N_0) / n_s
    Under flow, one FP32 FMA per nonzero entry of kappa for every bead and
    every spring's anchor: 0.5 flow_entries (1 + 1 / N_0) (flow_entries:
    nonzero entries of kappa, averaged over the beads).
    """
    return (37.5 + 18.75 + 4.5 + 10.5 + 1.5 / n0 + 24.0 / n0 + 1.0 + 4.5 / n0 + (9.0 + 9.0 / n0) / sample_every
            + 0.5 * flow_entries * (1.0 + 1.0 / n0))


# The step kernel's source and the headers it is compiled with.
KERNEL_SOURCES = ("ssp_step.hip", "ssp_device.h", "ssp_internal.h")


def kernel_sources_sha():
    """sha256 over the step kernel's source files, concatenated in order."""
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1106_2899_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def _traffic_from_profiles():
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when absent or taken on different kernel sources."""
    p = os.path.join(ROOT, "profiles", "step_kernel_lve_16384x32_counters.md")
    if not os.path.exists(p):
        return None
    d = {}
    with open(p) as f:
        for line in f:
            k, _, v = line.strip().partition(": ")
            if k in ("kernel_sources_sha256", "hbm_bytes_per_launch"):
                d[k] = v.strip()
    if d.get("kernel_sources_sha256") != kernel_sources_sha() or "hbm_bytes_per_launch" not in d:
        return None
    return float(d["hbm_bytes_per_launch"])


def headline(precision, md_steps, steps, warmup, keep=False):
    """(seconds for `steps` graph-replayed calls of md_steps steps, ensemble if keep)."""
    import torch

    from paper_1106_2899_amd.ensemble import Ensemble

    e = Ensemble(BEADS, CHAINS, precision=precision, seed=2, sample_every=SAMPLE_EVERY, corr_levels=16,
                 corr_batches=16, max_steps_per_launch=md_steps, use_graph=True)
    e.init()
    e.step(md_steps)  # first call captures the graph
    torch.cuda.synchronize()
    for _ in range(warmup):
        e.step(md_steps)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        e.step(md_steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    assert torch.isfinite(e.stress()).all()  # raises if a non-finite state was produced
    if keep:
        return t1 - t0, e
    e.close()
    return t1 - t0, None


def step_kernel_launch_ms(md_steps, launches):
    """Average step-kernel launch duration (HIP events on the launch stream)."""
    import torch

    from paper_1106_2899_amd.ensemble import Ensemble

    e = Ensemble(BEADS, CHAINS, precision="fp32", seed=2, sample_every=SAMPLE_EVERY, corr_levels=16,
                 corr_batches=16, max_steps_per_launch=md_steps, use_graph=False)
    e.init()
    e.step(md_steps)
    torch.cuda.synchronize()
    e.set_kernel_timing(True)
    for _ in range(launches):
        e.step(md_steps)
    ms, n, bead_steps = e.kernel_time()
    e.close()
    return ms / n, bead_steps / n


def equilibrium_fp64(steps=10_000, launch=1000):
    """Plain FP64 on the 64 x N = 8 equilibrium workload (sampled every step
    into the correlator), its full 1e4 steps; returns (result, ensemble)."""
    import torch

    from paper_1106_2899_amd import workloads
    from paper_1106_2899_amd.ensemble import Ensemble

    w = workloads.equilibrium_small()
    e = Ensemble(w.n_beads, precision="fp64", seed=w.seed, sample_every=1, corr_levels=16, corr_batches=8,
                 max_steps_per_launch=launch, use_graph=True).init()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e.step(steps)  # one graph launch of 10 chunks (includes the capture)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    return {"workload": w.name, "value": w.bead_steps / dt, "unit": "bead-steps/s", "steps": steps,
            "ms": dt * 1e3, "note": "latency-bound: 64 chains fill 2 % of the wavefront slots"}, e


def adjoint_ratio(chains=65536, beads=64, window=2000, ckpt=100, rate=0.01, reps=2):
    """Adjoint/forward time ratio on the differentiation workload: (recorded
    forward + reverse pass) / plain forward of the same window.  Two ways: a
    checkpoint every `ckpt` steps with each segment replayed in the reverse
    pass, and the window as one segment whose forward stores the trajectory
    (no replay; about 13 B of HBM per bead-step)."""
    import torch

    from paper_1106_2899_amd.ensemble import Ensemble

    kap = torch.zeros(1, 9, dtype=torch.float64, device="cuda")
    kap[0, 1] = rate
    e = Ensemble(beads, chains, precision="fp32", seed=5, sample_every=SAMPLE_EVERY, corr_levels=0, use_graph=True)
    e.init()
    e.step(window, kap)  # warm-up (graph capture)
    torch.cuda.synchronize()

    def timed(every):
        e.forward_record(window, every, kap)  # warm-up (buffer allocation)
        e.adjoint()
        torch.cuda.synchronize()
        t_fwd = t_rec = t_rev = 0.0
        for _ in range(reps):
            t0 = time.perf_counter()
            e.step(window, kap)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            e.forward_record(window, every, kap)
            torch.cuda.synchronize()
            t2 = time.perf_counter()
            g = e.adjoint()
            torch.cuda.synchronize()
            t3 = time.perf_counter()
            t_fwd += t1 - t0
            t_rec += t2 - t1
            t_rev += t3 - t2
        assert torch.isfinite(g).all()
        return {
            "checkpoint_every": every,
            "recording_GB": e._rec_bytes / 1e9,
            "forward_ms": t_fwd / reps * 1e3,
            "recorded_forward_ms": t_rec / reps * 1e3,
            "reverse_ms": t_rev / reps * 1e3,
            "adjoint_over_forward": (t_rec + t_rev) / t_fwd,
        }

    out = {"workload": f"adjoint_{chains}x{beads}", "window": window}
    out.update(timed(ckpt))
    try:
        out["stored_window"] = timed(window)
    except torch.OutOfMemoryError as err:
        out["stored_window"] = {"skipped": f"recording buffer does not fit: {err}"[:200]}
    e.close()
    torch.cuda.empty_cache()
    return out


def crn_fd_bias(chains=65536, beads=64, window=2000, rate=0.01, ns=0.5, h=1e-4):
    """The pathwise (event-conditioned) adjoint gradients of the ensemble mean
    of sigma_xy at the end of the window, d/d(shear rate) and d/dN_s, beside
    central finite differences of the free-running forward at rate +- h and
    N_s +- h on the same random streams (common random numbers), where slot
    decisions may flip.  The difference of the means is the stated bias of
    the pathwise gradient (it omits the jump contribution of the flipping
    decisions).  The perturbed runs advance in lock step with the unperturbed
    one, and a chain counts as flipped when its slot row differed at any step;
    over the other chains the per-chain differences must match the adjoint."""
    import numpy as np
    import torch

    from paper_1106_2899_amd.ensemble import Ensemble

    def kap(g):
        k = torch.zeros(1, 9, dtype=torch.float64, device="cuda")
        k[0, 1] = g
        return k

    params = {"base": (rate, ns), "rate-": (rate - h, ns), "rate+": (rate + h, ns), "ns-": (rate, ns - h),
              "ns+": (rate, ns + h)}

    def ens(n_s):
        return Ensemble(beads, chains, precision="fp32", seed=5, sample_every=SAMPLE_EVERY, corr_levels=0, ns=n_s,
                        use_graph=False).init()

    # pathwise gradients of the unperturbed window
    rec = ens(ns)
    rec.forward_record(window, 100, kap(rate))
    grad = rec.adjoint(component=3).cpu().numpy()
    S_rec = rec.state()[2]
    rec.close()
    runs = {k: ens(v[1]) for k, v in params.items()}
    kaps = {k: kap(v[0]) for k, v in params.items()}
    flipped = {k: torch.zeros(chains, dtype=torch.bool, device="cuda") for k in params if k != "base"}
    for _ in range(window):
        for k, e in runs.items():
            e.step(1, kaps[k])
        S0 = runs["base"].state()[2].view(chains, beads)
        for k in flipped:
            flipped[k] |= (runs[k].state()[2].view(chains, beads) != S0).any(dim=1)
    assert torch.equal(runs["base"].state()[2], S_rec)  # the recorded window is the unperturbed run
    J = {k: e.stress()[:, 3].cpu().numpy() for k, e in runs.items()}
    for e in runs.values():
        e.close()
    torch.cuda.empty_cache()
    out = {"workload": f"adjoint_{chains}x{beads}", "window": window, "h": h, "precision": "fp32"}
    for name, col, lo, hi in (("d_sigma_xy/d_rate", 1, "rate-", "rate+"), ("d_sigma_xy/d_ns", 9, "ns-", "ns+")):
        fd = (J[hi] - J[lo]) / (2 * h)
        kept = ~(flipped[lo] | flipped[hi]).cpu().numpy()
        adj = grad[:, col]
        rms = float(np.sqrt(np.mean(adj ** 2)))
        out[name] = {
            "adjoint_mean": float(adj.mean()),
            "crn_fd_mean": float(fd.mean()),
            "crn_fd_stderr": float(fd.std(ddof=1) / np.sqrt(chains)),
            "bias_adjoint_minus_fd": float(adj.mean() - fd.mean()),
            "chains_with_flipped_decisions": int((~kept).sum()),
            "unflipped_chains": {
                "adjoint_mean": float(adj[kept].mean()), "crn_fd_mean": float(fd[kept].mean()),
                "max_abs_diff_per_chain_over_rms": float(np.abs(adj[kept] - fd[kept]).max() / rms),
            } if kept.any() else None,
        }
    return out


def _flow_entries(w):
    """Nonzero entries of kappa per bead, averaged over the workload's beads."""
    import numpy as np

    nnz = (w.kappa.reshape(w.n_elements, 9) != 0).sum(axis=1)
    beads_per_elem = np.add.reduceat(w.n_beads.astype(np.int64), w.element_offsets[:-1])
    return float((nnz * beads_per_elem).sum() / beads_per_elem.sum())


def flow_workload(w, tune):
    """A flow workload at its full length: bead-steps/s of one graph-replayed
    ssp_step call of all its steps (after the call that captures the graph),
    and the step kernel's roofline fraction from HIP-event launch times of a
    1000-step call."""
    import torch

    from paper_1106_2899_amd import autotune
    from paper_1106_2899_amd.ensemble import Ensemble

    cap = w.steps // w.sample_every
    e = Ensemble(w.n_beads, n_elements=w.n_elements, element_offsets=w.element_offsets, precision="fp32",
                 seed=w.seed, sample_every=w.sample_every, corr_levels=0, series_capacity=cap, use_graph=True)
    kap = torch.as_tensor(w.kappa.reshape(w.n_elements, 9), dtype=torch.float64, device="cuda")
    tuned = None
    if tune:
        tuned = autotune.tune(e, w.kappa).to_json()
    e.init()
    e.step(w.steps, kap)  # graph capture and a full warm-up run
    torch.cuda.synchronize()
    e.init()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e.step(w.steps, kap)  # the whole run: one graph launch
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    assert torch.isfinite(e.stress()).all()
    bead_steps = int(w.n_beads.sum()) * w.steps
    e.set_kernel_timing(True)
    e.step(1000, kap)
    ms, n, bs = e.kernel_time()
    e.close()
    torch.cuda.empty_cache()
    rate_kernel = bs / (ms * 1e-3)
    slots = algorithmic_valu_slots(w.sample_every, flow_entries=_flow_entries(w))
    out = {"value": bead_steps / dt, "unit": "bead-steps/s", "steps": w.steps, "seconds": dt,
           "roofline": {"bound": "alu", "achieved": slots * rate_kernel, "peak": PEAK_LANE_SLOTS,
                        "unit": "VALU lane-slots/s", "frac": slots * rate_kernel / PEAK_LANE_SLOTS,
                        "algorithmic_slots_per_bead_step": slots, "kernel_bead_steps_per_s": rate_kernel}}
    if tuned:
        out["autotuned_mapping"] = json.loads(tuned)["choices"]
    return out


def _shear(rate):
    import numpy as np

    k = np.zeros((3, 3))
    k[0, 1] = rate
    return k


def paper_table_shapes():
    """Context rows: the shapes of the paper's timing table on this GPU (FP32,
    stress sampled every 10 steps, no correlator), each with the mapping the
    autotuner picks for it and run as one graph launch of all 1e4 steps after
    a warm-up run of the same length, beside the paper's GPU seconds.  65536
    beads fill a few percent of the wavefront slots, so these runs are
    latency-bound and carry no roofline."""
    import torch

    from paper_1106_2899_amd import autotune
    from paper_1106_2899_amd.ensemble import Ensemble

    rows = []
    for N, M, rate, paper_s in PAPER_TABLE_SHAPES:
        e = Ensemble(N, M, precision="fp32", seed=7, sample_every=SAMPLE_EVERY, corr_levels=0, use_graph=True)
        kap = None if rate == 0.0 else torch.as_tensor(_shear(rate).reshape(1, 9), dtype=torch.float64, device="cuda")
        mapping = json.loads(autotune.tune(e, kap).to_json())["choices"]
        e.init()
        e.step(PAPER_TABLE_STEPS, kap)  # graph capture and a full warm-up run
        torch.cuda.synchronize()
        e.init()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e.step(PAPER_TABLE_STEPS, kap)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        assert torch.isfinite(e.stress()).all()
        e.close()
        rows.append({"shape": f"{N}x{M}", "shear_rate": rate, "mapping": mapping, "steps": PAPER_TABLE_STEPS, "seconds": dt,
                     "value": N * M * PAPER_TABLE_STEPS / dt, "unit": "bead-steps/s",
                     "paper_gpu_seconds": paper_s, "speedup_over_paper_gpu": paper_s / dt})
    return rows


# ---------------------------------------------------------------- CPU leg --
# The FP64 oracle (test infrastructure) on the host cores: its timing, and
# the accuracy of every GPU number against it.

def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _lockstep_accuracy(ids, N, kchain, seed, steps, precision="fp32"):
    """Largest per-step error, relative to max(|x|, 0.58) (the tests' bar:
    1e-5 FP32, 1e-12 FP64), and the chains with a tie, of the chains `ids`
    advanced in lock step with the oracle from the same initial state."""
    import numpy as np
    import torch

    import oracle
    from paper_1106_2899_amd.ensemble import Ensemble

    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from _lockstep import lockstep

    M = len(ids)
    lengths = [int(N[i]) for i in ids]
    small = Ensemble(lengths, n_elements=M, element_offsets=np.arange(M + 1), chain_ids=np.asarray(ids, dtype=np.int64),
                     precision=precision, seed=seed, corr_levels=0).init()
    o = oracle.Ensemble(lengths, chain_ids=np.asarray(ids, dtype=np.int64), seed=seed).init()
    kc = None if kchain is None else np.ascontiguousarray(kchain[ids])
    ke = None if kc is None else torch.as_tensor(kc, dtype=torch.float64, device="cuda")
    fp64 = precision == "fp64"
    bar = 1e-12 if fp64 else 1e-5
    out = {"chains": M, "steps": steps, "bar": bar}
    try:
        st = lockstep(small, o, steps, kappa_elem=ke, kappa_chain=kc, tol=bar, fp64=fp64)
        out.update({"max_rel_error": st["worst"], "tie_chains": st["ties"], "within_bar": True})
    except AssertionError as err:
        out.update({"within_bar": False, "failure": str(err)[:300]})
    small.close()
    return out


def cpu_leg(G_gpu, steps_gpu, eq_ensemble, flow_ws):
    import numpy as np

    import oracle
    from paper_1106_2899_amd import workloads

    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from _corr import oracle_G

    oracle.build(force=False)
    n_all = oracle.threads()
    out = {}
    # all threads: the headline workload's first 1024 chains over the whole run
    sample_chains = 1024
    o = oracle.Ensemble([BEADS] * sample_chains, seed=2).init()
    t0 = time.perf_counter()
    s = o.run(steps_gpu, sample_every=SAMPLE_EVERY)
    dt = time.perf_counter() - t0
    baseline = {
        "value": sample_chains * BEADS * steps_gpu / dt,
        "unit": "bead-steps/s",
        "cores": n_all,
        "kind": "oracle",
        "sample": f"{sample_chains} chains x N={BEADS} x {steps_gpu} steps of the headline workload (its first "
                  f"chains, sampled every {SAMPLE_EVERY} steps), FP64, OpenMP over chains on {n_all} threads; "
                  f"{dt:.1f} s",
        "cpu_model": _cpu_model(),
        "affinity_cores": len(os.sched_getaffinity(0)),
    }
    # G(t) of the headline run against the oracle's, per lag, in units of the
    # two batch-means standard errors in quadrature (Sec. 2.3 Green-Kubo form)
    G, G_err, cnt = oracle_G(s, 16, batches=16)
    del s
    ok = cnt > 0
    sig = np.sqrt(G_gpu["G_err"] ** 2 + G_err ** 2)
    z = np.where(ok & (sig > 0), (G_gpu["G"] - G) / np.where(sig > 0, sig, 1.0), 0.0)
    _log(f"oracle on {n_all} threads: {baseline['value']:.4g} bead-steps/s")
    out["headline_G_t"] = {"lags": int(ok.sum()), "max_abs_z": float(np.abs(z[ok]).max()),
                           "rms_z": float(np.sqrt((z[ok] ** 2).mean())), "oracle_chains": sample_chains}
    # one thread: 64 chains of the headline workload for 1e4 steps
    oracle.set_threads(1)
    o1 = oracle.Ensemble([BEADS] * 64, seed=2).init()
    t0 = time.perf_counter()
    o1.run(10_000, sample_every=SAMPLE_EVERY, keep_samples=False)
    dt1 = time.perf_counter() - t0
    oracle.set_threads(n_all)
    baseline["one_thread"] = {"value": 64 * BEADS * 10_000 / dt1, "unit": "bead-steps/s", "cores": 1,
                              "sample": f"64 chains x N={BEADS} x 10000 steps, {dt1:.1f} s"}
    # accuracy: sampled chains of each workload in lock step with the oracle
    w2 = workloads.linear_viscoelasticity()
    ids = np.linspace(0, w2.n_chains - 1, 16).astype(np.int64)
    out["headline_fp32"] = _lockstep_accuracy(ids, w2.n_beads, None, w2.seed, 1000)
    out["same_shape_fp64"] = _lockstep_accuracy(ids[:8], w2.n_beads, None, w2.seed, 500, precision="fp64")
    for name, w in flow_ws:
        kchain = np.repeat(w.kappa.reshape(w.n_elements, 9), np.diff(w.element_offsets), axis=0)
        ids = np.linspace(0, w.n_chains - 1, 8).astype(np.int64)
        out[name] = _lockstep_accuracy(ids, w.n_beads, kchain, w.seed, 1000)
        _log(f"lock step {name} done")
    # the paper's timing-table shapes: the oracle in full at rest on all
    # threads, and sampled chains of the sheared extremes in lock step
    shapes = []
    for N, M, rate, _ in PAPER_TABLE_SHAPES:
        if rate != 0.0:
            continue
        o = oracle.Ensemble([N] * M, seed=7).init()
        t0 = time.perf_counter()
        o.run(PAPER_TABLE_STEPS, sample_every=SAMPLE_EVERY, keep_samples=False)
        dt = time.perf_counter() - t0
        shapes.append({"shape": f"{N}x{M}", "steps": PAPER_TABLE_STEPS, "seconds": dt, "threads": n_all,
                       "value": N * M * PAPER_TABLE_STEPS / dt, "unit": "bead-steps/s"})
    baseline["paper_table_shapes"] = shapes
    _log("oracle on the paper's table shapes done")
    for N, M in ((16, 4096), (128, 512)):
        ids = np.linspace(0, M - 1, 8).astype(np.int64)
        kchain = np.repeat(_shear(0.05).reshape(1, 9), M, axis=0)
        out[f"paper_shape_{N}x{M}_shear_0.05"] = _lockstep_accuracy(ids, np.full(M, N), kchain, 7, 1000)
    # the FP64 equilibrium run: final state of every chain after 1e4 steps
    if eq_ensemble is not None:
        w1 = workloads.equilibrium_small()
        R, A, S = (x.cpu().numpy() for x in eq_ensemble.state())
        o = oracle.Ensemble(w1.n_beads, seed=w1.seed).init()
        o.run(w1.steps, keep_samples=False)
        same = np.array_equal(S, o.S)
        M, N = w1.n_chains, int(w1.n_beads[0])
        b = (R.reshape(M, N, 3)[:, 1:] - R.reshape(M, N, 3)[:, :-1])
        bo = (o.R.reshape(M, N, 3)[:, 1:] - o.R.reshape(M, N, 3)[:, :-1])
        err = float((np.abs(b - bo) / np.maximum(np.abs(bo), 0.58)).max())
        out["equilibrium_fp64"] = {"decisions_identical": bool(same), "final_bond_max_rel_error": err,
                                   "steps": w1.steps, "bar": 1e-12}
    return baseline, out


def adjoint_accuracy(window=300, chains=8):
    """Per-chain FP32 gradients dJ/dkappa and dJ/dN_s of sampled chains of the
    differentiation workload (one stored window) against the oracle's adjoint
    of its own forward, each column relative to its largest entry (the
    tests' measure), when both took the same slot decisions."""
    import numpy as np
    import torch

    import oracle
    from paper_1106_2899_amd import workloads
    from paper_1106_2899_amd.ensemble import Ensemble

    w = workloads.differentiation()
    ids = np.linspace(0, w.n_chains - 1, chains).astype(np.int64)
    lengths = [int(w.n_beads[i]) for i in ids]
    kap = w.kappa.reshape(1, 9)
    e = Ensemble(lengths, chain_ids=ids, precision="fp32", seed=w.seed, corr_levels=0).init()
    e.forward_record(window, window, kap)
    got = e.adjoint(component=3).cpu().numpy()
    S_end = e.state()[2].cpu().numpy()
    e.close()
    o = oracle.Ensemble(lengths, chain_ids=ids, seed=w.seed).init()
    Rt, At, St = o.run_record(window, kap)
    gk, gns = o.adjoint(Rt, At, St, kap, comp=3)
    want = np.concatenate([gk.reshape(chains, 9), gns[:, None]], axis=1)
    scale = np.abs(want).max(axis=0)
    scale[scale == 0] = 1.0
    torch.cuda.empty_cache()
    out = {"chains": chains, "window": window, "events_identical": bool(np.array_equal(S_end, o.S)), "bar": 1e-4}
    if out["events_identical"]:
        out["max_rel_error"] = float((np.abs(got - want) / scale).max())
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the step path runs on a single MI355X (--gpus 1); sharding across GPUs is described, not built.", file=sys.stderr)
        sys.exit(2)

    import torch

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(2)

    from paper_1106_2899_amd import workloads

    md = MD_STEPS_PER_BENCH_STEP
    beads = CHAINS * BEADS
    # batched FP32 (headline), graph replay; the ensemble is kept for its G(t)
    t32, e32 = headline("fp32", md, args.steps, args.warmup, keep=True)
    v32 = beads * md * args.steps / t32
    _log(f"fp32 headline: {v32:.4g} bead-steps/s")
    G_gpu = e32.correlator()
    steps_gpu = e32.steps
    e32.close()
    # plain FP64 at the same shape (fewer steps: same per-step work, slower path)
    k64 = max(2, args.steps // 4)
    t64, _ = headline("fp64", md, k64, 1)
    v64 = beads * md * k64 / t64
    _log(f"fp64 same shape: {v64:.4g} bead-steps/s")
    # roofline leg: step-kernel launch durations from HIP events on the launch stream
    launch_ms, bead_steps = step_kernel_launch_ms(md, max(3, args.steps // 4))
    slots = algorithmic_valu_slots()
    achieved = slots * bead_steps / (launch_ms * 1e-3)
    roofline = {
        "bound": "alu",
        "kernel": QUEUE_KERNEL,
        "achieved": achieved,
        "peak": PEAK_LANE_SLOTS,
        "unit": "VALU lane-slots/s",
        "frac": achieved / PEAK_LANE_SLOTS,
        "traffic": _traffic_from_profiles(),
        "algorithmic_slots_per_bead_step": slots,
        "launch_ms": launch_ms,
        "bead_steps_per_launch": bead_steps,
    }
    _log(f"roofline frac {roofline['frac']:.3f}")
    eq, eq_ens = equilibrium_fp64()
    _log("fp64 equilibrium 64x8 done")
    flow_ws = [("startup_shear_4096x256x32", workloads.startup_shear()), ("polydisperse_2^18", workloads.polydisperse())]
    out = {
        "metric": "bead-steps/sec on 1 MI355X (batched FP32 vs plain FP64); adjoint/forward time ratio",
        "value": v32,
        "unit": "bead-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t32 / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "lve_16384x32",
            "chains": CHAINS,
            "beads": BEADS,
            "time_steps_per_bench_step": md,
            "sample_every": SAMPLE_EVERY,
            "correlator": "multiple-tau 16x16 FP64",
            "n0": 4.0, "ns": 0.5, "zeta_s": 0.1, "dt": 0.01,
        },
        "fp64_plain": {"value": v64, "unit": "bead-steps/s", "steps": k64, "ms_per_step": t64 / k64 * 1e3,
                       "workload": "lve_16384x32 (same shape)"},
        "fp32_over_fp64": v32 / v64,
        "fp64_equilibrium_64x8": eq,
        "roofline": roofline,
    }
    out["adjoint"] = adjoint_ratio()
    _log(f"adjoint/forward {out['adjoint']['adjoint_over_forward']:.3f}")
    out["adjoint_crn_fd"] = crn_fd_bias()
    _log("adjoint vs free-running CRN finite differences done")
    out["flow_workloads"] = {}
    for name, w in flow_ws:
        out["flow_workloads"][name] = flow_workload(w, tune=name.startswith("poly"))
        _log(f"{name}: {out['flow_workloads'][name]['value']:.4g} bead-steps/s")
    out["paper_table_shapes"] = paper_table_shapes()
    _log("paper's table shapes done")
    if not args.no_cpu_baseline:
        baseline, acc = cpu_leg(G_gpu, steps_gpu, eq_ens, flow_ws)
        acc["adjoint_stored_window"] = adjoint_accuracy()
        out["cpu_baseline"] = baseline
        out["accuracy_vs_oracle"] = acc
    eq_ens.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
