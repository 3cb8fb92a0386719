"""Benchmark of the slip-spring ensemble step on one MI355X.

Workload: the equilibrium linear-viscoelasticity ensemble, 16384 chains of
N = 32 beads (N_0 = 4, N_s = 0.5, zeta_s = 0.1, dt = 0.01), FP32 bead dynamics
with FP64 stress, stress sampled every 10 steps into the FP64 multiple-tau
correlator (16 levels x 16 lags).  One benchmark step is one ssp_step call of
5000 time steps over the whole ensemble (every row of the hot path: RNG,
forces, Euler move, hops, reconstruction, stress, correlator), replayed from a
captured hipGraph; the default 20 steps are the full 1e5-step run.  Inputs are
resident in HBM before the timed region.

Printed: one JSON line with bead-steps/s of the batched FP32 path, the plain
FP64 path at the same shape, the VALU roofline of the step kernel (measured
with HIP events on the launch stream), the adjoint/forward time ratio (a
checkpoint every 100 steps, and the window stored as one segment), the
batched FP32 path on the start-up shear and polydisperse workloads (context),
and the FP64 CPU oracle timed on the host cores on a bounded sample.
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


def algorithmic_valu_slots(sample_every: int = SAMPLE_EVERY, n0: float = 4.0) -> float:
    """VALU lane-issue slots per bead-step that the method needs on this
    workload (kappa = 0), each operation weighted by its issue cost measured
    on gfx950 with a throughput probe (full rate = 1, which includes the
    32x32->64 integer multiply, the three-input bitop and FP64 FMA; FP32
    transcendentals log/exp/sin/cos/sqrt/rcp = 2), in the arithmetic the path
    requires (compensated FP32 positions) and with the random stream at its
    minimum of five words per bead-step:
      random words: 1.5 Box-Muller pairs (3 words) + hop + reconstruction
        = 1.25 Philox4x32-10 blocks x 10 rounds x (2 products + 2 xors)  ->  50
      Box-Muller, 1.5 pairs x (2 uniforms x 2, log 2, mul, sqrt 2,
        sin 2, cos 2, 2 mul)                                           ->  22.5
      bonds from compensated positions, 3 x 3                          ->   9
      move: bond-force difference 3, two FMAs per component 6,
        compensated position update 12                                 ->  21
      spring-force gather, 3 adds per spring                           ->   3 / N_0
      hop per occupied slot: post-move offset 3, two energy
        differences 12, two probabilities 2 x 8, decision 5            ->  36 / N_0
      reconstruction word test                                         ->   2
      anchor offsets for the next step (compensated), per spring      ->   9 / N_0
      stress and virtual stress (FP64), per sample: per bead 3 cvt
        + 6 FMA, per spring the same                                   ->  (9 + 9 / N_0) / n_s
    """
    return 50.0 + 22.5 + 9.0 + 21.0 + 3.0 / n0 + 36.0 / n0 + 2.0 + 9.0 / n0 + (9.0 + 9.0 / n0) / sample_every


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


def run_gpu(precision, md_steps, steps, warmup, timing=False, use_graph=True):
    import torch

    from paper_1106_2899_amd.ensemble import Ensemble

    e = Ensemble(BEADS, CHAINS, precision=precision, seed=2, sample_every=SAMPLE_EVERY, corr_levels=16,
                 corr_batches=16, max_steps_per_launch=md_steps, use_graph=use_graph)
    e.init()
    e.step(md_steps)  # first call captures the graph
    torch.cuda.synchronize()
    if timing:
        e.set_kernel_timing(True)
    for _ in range(warmup):
        e.step(md_steps)
    torch.cuda.synchronize()
    if timing:
        e.kernel_time()  # discard warm-up launches
    t0 = time.perf_counter()
    for _ in range(steps):
        e.step(md_steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kt = e.kernel_time() if timing else None
    stress = e.stress()  # raises if a non-finite state was produced
    assert torch.isfinite(stress).all()
    e.close()
    return t1 - t0, kt


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


def batched_configs(md_steps=1000, launches=3):
    """Context, not the headline: bead-steps/s of the batched FP32 path on the
    two flow workloads at their full sizes, timed over `launches` graph-replayed
    calls of `md_steps` steps after one warm-up call (fewer steps than the
    workloads' full runs; per-step work is the same).
      startup_shear_4096x256x32: 1,048,576 chains of N = 32 in 4096 elements,
        each sheared at its own rate, element series sampled every 10 steps;
      polydisperse_2^18: 262,144 chains, N uniform in 16..128, shear or
        uniaxial elongation per element, mapping chosen by the autotuner."""
    import torch

    from paper_1106_2899_amd import autotune, workloads
    from paper_1106_2899_amd.ensemble import Ensemble

    out = {}
    for w, tune in ((workloads.startup_shear(), False), (workloads.polydisperse(), True)):
        cap = (launches + 1) * md_steps // w.sample_every
        e = Ensemble(w.n_beads, n_elements=w.n_elements, element_offsets=w.element_offsets, precision="fp32",
                     seed=w.seed, sample_every=w.sample_every, corr_levels=0, series_capacity=cap,
                     max_steps_per_launch=md_steps, use_graph=True)
        if tune:
            autotune.tune(e, w.kappa)
        e.init()
        kap = torch.as_tensor(w.kappa.reshape(w.n_elements, 9), dtype=torch.float64, device="cuda")
        e.step(md_steps, kap)  # graph capture and warm-up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(launches):
            e.step(md_steps, kap)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        assert torch.isfinite(e.stress()).all()  # raises on a latched non-finite state
        e.close()
        out[w.name] = {"value": int(w.n_beads.sum()) * md_steps * launches / dt, "unit": "bead-steps/s",
                       "steps": md_steps * launches}
    return out


def cpu_baseline(sample_chains=4096, sample_steps=16000):
    import oracle

    oracle.build(force=False)
    o = oracle.Ensemble([BEADS] * sample_chains, seed=2).init()
    t0 = time.perf_counter()
    o.run(sample_steps, sample_every=SAMPLE_EVERY, keep_samples=False)
    dt = time.perf_counter() - t0
    return {
        "value": sample_chains * BEADS * sample_steps / dt,
        "unit": "bead-steps/s",
        "cores": oracle.threads(),
        "kind": "oracle",
        "sample": f"{sample_chains} chains x N={BEADS} x {sample_steps} steps of the same workload "
                  f"(sampling every {SAMPLE_EVERY} steps), FP64, OpenMP over chains; {dt:.1f} s",
    }


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

    md = MD_STEPS_PER_BENCH_STEP
    beads = CHAINS * BEADS
    # batched FP32 (headline), graph replay
    t32, _ = run_gpu("fp32", md, args.steps, args.warmup)
    v32 = beads * md * args.steps / t32
    # plain FP64 at the same shape (fewer steps: same per-step work, slower path)
    k64 = max(2, args.steps // 4)
    t64, _ = run_gpu("fp64", md, k64, 1)
    v64 = beads * md * k64 / t64
    # roofline leg: step-kernel launch durations from HIP events on the launch stream
    _, (ms, launches, bead_steps) = run_gpu("fp32", md, max(3, args.steps // 4), 1, timing=True, use_graph=False)
    per_launch_s = ms / 1e3 / launches
    slots = algorithmic_valu_slots()
    achieved = slots * (bead_steps / launches) / per_launch_s
    roofline = {
        "bound": "alu",
        "kernel": "k_step<float,32,1,false,false>",
        "achieved": achieved,
        "peak": PEAK_LANE_SLOTS,
        "unit": "VALU lane-slots/s",
        "frac": achieved / PEAK_LANE_SLOTS,
        "traffic": _traffic_from_profiles(),
        "algorithmic_slots_per_bead_step": slots,
        "launch_ms": per_launch_s * 1e3,
        "bead_steps_per_launch": bead_steps / launches,
    }
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
        "fp64_plain": {"value": v64, "unit": "bead-steps/s", "steps": k64, "ms_per_step": t64 / k64 * 1e3},
        "fp32_over_fp64": v32 / v64,
        "roofline": roofline,
        "adjoint": adjoint_ratio(),
        "batched_configs": batched_configs(),
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
