"""Short, fixed GPU runs for rocprofv3 (kernel trace and counter passes).

    python -m paper_1106_2899_amd.profile_run step   # step kernel, 16384 x N=32, 3 launches of 5000 steps
    python -m paper_1106_2899_amd.profile_run flow   # the same ensemble under simple shear (rate 1) and under
                                                     # uniaxial elongation (rate 0.05), 2 launches of 2000 steps each
    python -m paper_1106_2899_amd.profile_run copy   # 1 GiB read + 1 GiB write elementwise copy (counter calibration)
    python -m paper_1106_2899_amd.profile_run adjoint  # 65536 x N=64 under shear 0.01: forward, recorded forward, reverse
    python -m paper_1106_2899_amd.profile_run adjoint_stored  # the same window as one stored segment (no replay)
    python -m paper_1106_2899_amd.profile_run issue    # VALU issue cost per instruction kind (libssp_probe.so)
"""
from __future__ import annotations

import sys

import torch


def step(launches: int = 3, md_steps: int = 5000) -> None:
    from .ensemble import Ensemble

    e = Ensemble(32, 16384, precision="fp32", seed=2, sample_every=10, corr_levels=16, corr_batches=16,
                 max_steps_per_launch=md_steps, use_graph=False)
    e.init()
    for _ in range(launches):
        e.step(md_steps)
    torch.cuda.synchronize()
    print("step launches:", launches, "bead-steps per launch:", 16384 * 32 * md_steps, flush=True)


def flow(launches: int = 2, md_steps: int = 2000) -> None:
    from .ensemble import Ensemble

    for name, kap in (("shear 1.0", [0, 1.0, 0, 0, 0, 0, 0, 0, 0]),
                      ("elongation 0.05", [0.05, 0, 0, 0, -0.025, 0, 0, 0, -0.025])):
        e = Ensemble(32, 16384, precision="fp32", seed=2, sample_every=10, corr_levels=16, corr_batches=16,
                     max_steps_per_launch=md_steps, use_graph=False)
        e.init()
        k = torch.tensor(kap, dtype=torch.float64, device="cuda").reshape(1, 9)
        for _ in range(launches):
            e.step(md_steps, k)
        torch.cuda.synchronize()
        e.close()
        print("flow", name, "launches:", launches, "bead-steps per launch:", 16384 * 32 * md_steps, flush=True)


def adjoint(chains: int = 65536, beads: int = 64, window: int = 2000, ckpt: int = 100, rate: float = 0.01) -> None:
    from .ensemble import Ensemble

    kap = torch.zeros(1, 9, dtype=torch.float64, device="cuda")
    kap[0, 1] = rate
    e = Ensemble(beads, chains, precision="fp32", seed=5, sample_every=10, corr_levels=0, use_graph=False)
    e.init()
    e.step(window, kap)
    e.forward_record(window, ckpt, kap)
    g = e.adjoint()
    torch.cuda.synchronize()
    assert torch.isfinite(g).all()
    print("adjoint window:", window, "checkpoint every:", ckpt, "bead-steps per pass:", chains * beads * window, flush=True)


def adjoint_stored() -> None:
    adjoint(ckpt=2000)


def copy(nbytes: int = 1 << 30) -> None:
    a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    torch.mul(a, 1.0, out=b)  # reads nbytes, writes nbytes
    torch.cuda.synchronize()
    print("copy bytes read:", nbytes, "written:", nbytes, flush=True)


def issue(iters: int = 16000, waves_per_simd: int = 8) -> None:
    """One launch per VALU instruction kind of the probe library: every SIMD
    runs `waves_per_simd` waves of 32 x iters independent instructions of the
    kind.  Prints the launch times (HIP events) and nanoseconds per
    instruction and SIMD; the cost in SIMD cycles comes from the same run
    under rocprofv3 (GRBM_GUI_ACTIVE per XCD over SQ_INSTS_VALU / SIMDs)."""
    import ctypes
    import os

    lib = ctypes.CDLL(os.path.join(os.path.dirname(os.path.abspath(__file__)), "libssp_probe.so"))
    lib.ssp_probe_name.restype = ctypes.c_char_p
    lib.ssp_probe_run.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p,
                                  ctypes.POINTER(ctypes.c_float)]
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    blocks = cus * waves_per_simd  # 4 waves per workgroup, 4 SIMDs per CU
    sink = torch.empty(blocks * 256, dtype=torch.float32, device="cuda")
    ms = ctypes.c_float()
    per_simd = 32 * iters * waves_per_simd
    print(f"CUs {cus}, {waves_per_simd} waves per SIMD, {per_simd} instructions per SIMD", flush=True)
    print("| Instruction | launch ms | ns per instruction and SIMD |")
    print("|---|---|---|")
    for op in range(lib.ssp_probe_count()):
        for it in (16, iters):  # a short warm-up launch, then the measured one
            if lib.ssp_probe_run(op, blocks, it, ctypes.c_void_p(sink.data_ptr()), ctypes.byref(ms)) != 0:
                raise RuntimeError(f"probe {op} failed")
        print(f"| {lib.ssp_probe_name(op).decode()} | {ms.value:.3f} | {ms.value * 1e6 / per_simd:.3f} |", flush=True)


if __name__ == "__main__":
    {"step": step, "flow": flow, "copy": copy, "adjoint": adjoint, "adjoint_stored": adjoint_stored,
     "issue": issue}[sys.argv[1]]()
