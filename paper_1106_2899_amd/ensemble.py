"""Python binding of libssp: an ensemble of slip-spring chains on one GPU.

PyTorch provides device memory and streams; all arithmetic of the method runs
in the HIP library behind the C ABI of include/ssp.h.
"""
from __future__ import annotations

import ctypes
import warnings
from typing import Optional, Sequence, Union

import numpy as np
import torch

from . import _lib
from ._lib import SspConfig, check, lib

_ALIGN = 256


def _aligned_buffer(nbytes: int, device) -> tuple[torch.Tensor, int]:
    t = torch.empty(max(int(nbytes), 1) + _ALIGN, dtype=torch.uint8, device=device)
    p = t.data_ptr()
    return t, (p + _ALIGN - 1) // _ALIGN * _ALIGN


class Ensemble:
    """An ensemble of independent single-chain slip-spring chains.

    Parameters follow the paper's notation: N beads per chain (scalar or per
    chain), N_0 (mean spacing of slip-springs, <Z> = N/N_0), N_s (slip-spring
    strength), zeta_s (slip-spring friction), dt.  Chains are grouped into
    elements (contiguous chain ranges), each with its own velocity gradient.
    """

    def __init__(
        self,
        n_beads: Union[int, Sequence[int]],
        n_chains: Optional[int] = None,
        *,
        n_elements: int = 1,
        element_offsets: Optional[Sequence[int]] = None,
        chain_ids: Optional[Sequence[int]] = None,
        precision: str = "fp32",
        sample_every: int = 1,
        dt: float = 0.01,
        n0: float = 4.0,
        ns: float = 0.5,
        zeta_s: float = 0.1,
        seed: int = 1,
        corr_levels: int = 16,
        corr_batches: int = 16,
        series_capacity: int = 0,
        max_steps_per_launch: int = 0,
        use_graph: bool = True,
        construct_rule: int = 0,
        corr_virtual: bool = False,
        device: Union[str, torch.device, None] = None,
        stream: Optional[torch.cuda.Stream] = None,
    ):
        L = lib()
        self.device = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        if self.device.type != "cuda":
            raise ValueError("the ensemble lives on a GPU device")
        if np.ndim(n_beads) == 0:
            if n_chains is None:
                raise ValueError("n_chains is required when n_beads is a scalar")
            self.N = np.full(int(n_chains), int(n_beads), dtype=np.int32)
        else:
            self.N = np.ascontiguousarray(n_beads, dtype=np.int32)
        self.M = int(self.N.shape[0])
        self.n_elements = int(n_elements)
        self.precision = precision
        cfg = SspConfig()
        L.ssp_config_init(ctypes.byref(cfg))
        cfg.n_chains = self.M
        cfg.n_elements = self.n_elements
        cfg.precision = {"fp32": _lib.SSP_FP32, "fp64": _lib.SSP_FP64}[precision]
        self._N_host = self.N
        cfg.n_beads_host = self._N_host.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        cfg.sample_every = int(sample_every)
        if element_offsets is not None:
            self.element_offsets = np.ascontiguousarray(element_offsets, dtype=np.int32)
            cfg.element_offsets_host = self.element_offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        else:
            self.element_offsets = (np.arange(self.n_elements + 1, dtype=np.int64) * self.M // self.n_elements).astype(np.int32)
        if chain_ids is not None:
            self._ids = np.ascontiguousarray(chain_ids, dtype=np.int64)
            cfg.chain_ids_host = self._ids.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))
            self.chain_ids = self._ids
        else:
            self.chain_ids = np.arange(self.M, dtype=np.int64)
        cfg.dt, cfg.n0, cfg.ns, cfg.zeta_s = float(dt), float(n0), float(ns), float(zeta_s)
        cfg.seed = int(seed)
        cfg.corr_levels = int(corr_levels)
        cfg.corr_batches = int(min(corr_batches, self.M)) if corr_levels else int(corr_batches)
        cfg.series_capacity = int(series_capacity)
        cfg.max_steps_per_launch = int(max_steps_per_launch)
        cfg.use_graph = 1 if use_graph else 0
        cfg.construct_rule = int(construct_rule)  # 0: K = C - Z, 1: K = 1 (Sec. 3.2)
        cfg.corr_virtual = 1 if corr_virtual else 0
        self.cfg = cfg
        self.dt, self.n0, self.ns, self.zeta_s, self.seed = cfg.dt, cfg.n0, cfg.ns, cfg.zeta_s, cfg.seed
        self.sample_every = cfg.sample_every
        self.corr_levels = cfg.corr_levels
        self.series_capacity = cfg.series_capacity
        sb, wb = ctypes.c_size_t(), ctypes.c_size_t()
        check(L.ssp_query_sizes(ctypes.byref(cfg), ctypes.byref(sb), ctypes.byref(wb)))
        msg = L.ssp_warning(None)
        if msg:
            warnings.warn(msg.decode(), stacklevel=2)
        self.state_bytes, self.work_bytes = sb.value, wb.value
        with torch.cuda.device(self.device):
            self._state_t, self._state_p = _aligned_buffer(sb.value, self.device)
            self._work_t, self._work_p = _aligned_buffer(wb.value, self.device)
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            h = ctypes.c_void_p()
            check(L.ssp_create(ctypes.byref(cfg), ctypes.c_void_p(self._state_p), ctypes.c_void_p(self._work_p),
                               ctypes.byref(h)))
        self._h = h
        self.total_beads = int(self.N.sum())
        self.offsets = np.zeros(self.M, dtype=np.int64)
        if self.M > 1:
            self.offsets[1:] = np.cumsum(self.N[:-1], dtype=np.int64)
        self._zero_kappa = torch.zeros((self.n_elements, 9), dtype=torch.float64, device=self.device)

    # ---------------------------------------------------------------- util
    @property
    def _s(self):
        return ctypes.c_void_p(self.stream.cuda_stream)

    def _chk(self, rc):
        check(rc, self._h)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().ssp_destroy(self._h)
            self._h = ctypes.c_void_p()
        self._rec_t, self._rec_bytes = None, 0  # the recording buffer can be most of the device

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------- methods
    def init(self) -> "Ensemble":
        """Equilibrium initial state (Sec. 3.1 sampling procedure)."""
        self._chk(lib().ssp_init_equilibrium(self._h, self._s))
        return self

    def kappa_tensor(self, kappa) -> torch.Tensor:
        """[E][9] FP64 device tensor of velocity gradients (row-major 3x3)."""
        if kappa is None:
            return self._zero_kappa
        k = torch.as_tensor(kappa, dtype=torch.float64, device=self.device)
        if k.numel() == 9:
            k = k.reshape(1, 9).expand(self.n_elements, 9)
        k = k.reshape(self.n_elements, 9).contiguous()
        return k

    def _kappa_arg(self, kappa):
        """(device table or None, pointer): None is a run at rest (the library's
        variant without flow terms; the same trajectory as a zero table)."""
        if kappa is None:
            return None, ctypes.c_void_p(None)
        k = self.kappa_tensor(kappa)
        return k, ctypes.c_void_p(k.data_ptr())

    def step(self, n_steps: int, kappa=None) -> "Ensemble":
        """Advance n_steps steps under velocity gradient kappa (per element; None: at rest)."""
        k, kp = self._kappa_arg(kappa)
        self._last_kappa = k  # keep alive while the stream may still read it
        self._chk(lib().ssp_step(self._h, int(n_steps), kp, self._s))
        return self

    @property
    def steps(self) -> int:
        v = ctypes.c_int64()
        self._chk(lib().ssp_step_count(self._h, ctypes.byref(v)))
        return v.value

    def stress(self) -> torch.Tensor:
        """[M][12] FP64: sigma (xx yy zz xy yz zx) then sigma^v."""
        out = torch.empty((self.M, 12), dtype=torch.float64, device=self.device)
        self._chk(lib().ssp_read_stress(self._h, ctypes.c_void_p(out.data_ptr()), self._s))
        return out

    def element_stress(self) -> torch.Tensor:
        """[E][12] FP64: the mean over each element's chains of sigma then sigma^v."""
        out = torch.empty((self.n_elements, 12), dtype=torch.float64, device=self.device)
        self._chk(lib().ssp_read_element_stress(self._h, ctypes.c_void_p(out.data_ptr()), self._s))
        return out

    def step_count(self) -> int:
        """Steps completed since init()."""
        n = ctypes.c_int64()
        self._chk(lib().ssp_step_count(self._h, ctypes.byref(n)))
        return int(n.value)

    def state(self):
        """Canonical FP64 state: R [sumN,3], A [sumN,3], S [sumN] (-1 = empty slot)."""
        R = torch.empty((self.total_beads, 3), dtype=torch.float64, device=self.device)
        A = torch.empty((self.total_beads, 3), dtype=torch.float64, device=self.device)
        S = torch.empty((self.total_beads,), dtype=torch.int32, device=self.device)
        self._chk(lib().ssp_read_state(self._h, ctypes.c_void_p(R.data_ptr()), ctypes.c_void_p(A.data_ptr()),
                                       ctypes.c_void_p(S.data_ptr()), self._s))
        return R, A, S

    def write_state(self, R, A, S) -> "Ensemble":
        R = torch.as_tensor(R, dtype=torch.float64, device=self.device).reshape(self.total_beads, 3).contiguous()
        A = torch.as_tensor(A, dtype=torch.float64, device=self.device).reshape(self.total_beads, 3).contiguous()
        S = torch.as_tensor(S, dtype=torch.int32, device=self.device).reshape(self.total_beads).contiguous()
        self._chk(lib().ssp_write_state(self._h, ctypes.c_void_p(R.data_ptr()), ctypes.c_void_p(A.data_ptr()),
                                        ctypes.c_void_p(S.data_ptr()), self._s))
        self.stream.synchronize()
        return self

    def element_series(self) -> torch.Tensor:
        """[E][T][6] per-element sums of sigma (xx yy zz xy yz zx) per sample."""
        out = torch.empty((self.n_elements, self.series_capacity, 6), dtype=torch.float64, device=self.device)
        n = ctypes.c_int64()
        self._chk(lib().ssp_read_element_series(self._h, ctypes.c_void_p(out.data_ptr()), ctypes.byref(n), self._s))
        return out[:, : n.value]

    def correlator(self):
        """Multiple-tau Green-Kubo correlator: dict(tau, G, G_err, counts), [levels*16] each."""
        L = self.corr_levels
        G = torch.empty(L * 16, dtype=torch.float64, device=self.device)
        E = torch.empty(L * 16, dtype=torch.float64, device=self.device)
        tau = np.zeros(L * 16)
        cnt = np.zeros(L * 16, dtype=np.int64)
        self._chk(lib().ssp_read_correlator(self._h, ctypes.c_void_p(G.data_ptr()), ctypes.c_void_p(E.data_ptr()),
                                            tau.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                            cnt.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), self._s))
        return {"tau": tau.reshape(L, 16), "G": G.cpu().numpy().reshape(L, 16),
                "G_err": E.cpu().numpy().reshape(L, 16), "counts": cnt.reshape(L, 16)}

    def correlator_virtual(self):
        """Virtual-stress channel: dict(tau, Gv, Gv_err) with
        Gv = <sigma^v(t) [sigma + sigma^v](0)>, and dG_v = Gv / G, the relative
        contribution of the virtual stress (Sec. 4.1), where G != 0."""
        L = self.corr_levels
        Gv = torch.empty(L * 16, dtype=torch.float64, device=self.device)
        E = torch.empty(L * 16, dtype=torch.float64, device=self.device)
        R = torch.empty(L * 16, dtype=torch.float64, device=self.device)
        self._chk(lib().ssp_read_correlator_virtual(self._h, ctypes.c_void_p(Gv.data_ptr()), ctypes.c_void_p(E.data_ptr()),
                                                    ctypes.c_void_p(R.data_ptr()), self._s))
        c = self.correlator()
        return {"tau": c["tau"], "Gv": Gv.cpu().numpy().reshape(L, 16), "Gv_err": E.cpu().numpy().reshape(L, 16),
                "counts": c["counts"], "dG_v": R.cpu().numpy().reshape(L, 16)}

    def linear_viscoelasticity(self, omega, t_lo: float, t_hi: float, G=None):
        """G'(w), G''(w), |eta*(w)|, eta_0 and tau_d from the relaxation modulus
        (Sec. 4.1 relations), computed on the device; G defaults to the
        correlator's current G(t) ([levels*16] FP64 on the device)."""
        if G is None:
            G = torch.as_tensor(self.correlator()["G"].ravel(), dtype=torch.float64, device=self.device)
        G = G.to(device=self.device, dtype=torch.float64).contiguous()
        w = torch.as_tensor(np.asarray(omega, dtype=np.float64), device=self.device).contiguous()
        moduli = torch.empty((w.numel(), 3), dtype=torch.float64, device=self.device)
        scalars = torch.empty(2, dtype=torch.float64, device=self.device)
        self._chk(lib().ssp_linear_viscoelasticity(self._h, ctypes.c_void_p(G.data_ptr()), ctypes.c_void_p(w.data_ptr()),
                                                   int(w.numel()), float(t_lo), float(t_hi),
                                                   ctypes.c_void_p(moduli.data_ptr()),
                                                   ctypes.c_void_p(scalars.data_ptr()), self._s))
        m, sc = moduli.cpu().numpy(), scalars.cpu().numpy()
        return {"omega": w.cpu().numpy(), "Gp": m[:, 0], "Gpp": m[:, 1], "eta_abs": m[:, 2],
                "eta0": float(sc[0]), "tau_d": float(sc[1])}

    def reset_observables(self) -> "Ensemble":
        self._chk(lib().ssp_reset_observables(self._h, self._s))
        return self

    def rng_normals(self, chain_id: int, step: int, bead: int, count: int) -> torch.Tensor:
        out = torch.empty((count, 3), dtype=torch.float64, device=self.device)
        self._chk(lib().ssp_rng_normals(self._h, int(chain_id), int(step), int(bead), int(count),
                                        ctypes.c_void_p(out.data_ptr()), self._s))
        self.stream.synchronize()
        return out

    # ----------------------------------------------------- differentiation
    def forward_record(self, window: int, ckpt_every: int, kappa=None) -> "Ensemble":
        """Advance `window` steps (like step) while recording what the adjoint needs."""
        nbytes = ctypes.c_size_t()
        self._chk(lib().ssp_adjoint_bytes(self._h, int(window), int(ckpt_every), ctypes.byref(nbytes)))
        if getattr(self, "_rec_bytes", 0) < nbytes.value:
            self._rec_t = None
            with torch.cuda.device(self.device):
                self._rec_t, self._rec_p = _aligned_buffer(nbytes.value, self.device)
            self._rec_bytes = nbytes.value
        k, kp = self._kappa_arg(kappa)
        self._rec_kappa, self._rec_kappa_p = k, kp
        self._chk(lib().ssp_forward_record(self._h, int(window), int(ckpt_every), kp,
                                           ctypes.c_void_p(self._rec_p), self._s))
        return self

    def adjoint(self, component: int = 3, init_window: bool = True) -> torch.Tensor:
        """[M][10] FP64: dJ_k/dkappa (9, row-major) and dJ_k/dN_s for J_k = the
        final stress component of chain k over the last recorded window."""
        out = torch.empty((self.M, 10), dtype=torch.float64, device=self.device)
        self._chk(lib().ssp_adjoint(self._h, ctypes.c_void_p(self._rec_p), self._rec_kappa_p,
                                    int(component), 1 if init_window else 0, ctypes.c_void_p(out.data_ptr()), self._s))
        return out

    def adjoint_elements(self, component: int = 3, init_window: bool = True):
        """(elem [E][10], chain [M][10]) FP64: the per-element means (library
        reduction) and the per-chain values of dJ_k/dkappa (9) and dJ_k/dN_s."""
        chain = torch.empty((self.M, 10), dtype=torch.float64, device=self.device)
        elem = torch.empty((self.n_elements, 10), dtype=torch.float64, device=self.device)
        self._chk(lib().ssp_adjoint_elements(self._h, ctypes.c_void_p(self._rec_p), self._rec_kappa_p, int(component),
                                             1 if init_window else 0, ctypes.c_void_p(chain.data_ptr()),
                                             ctypes.c_void_p(elem.data_ptr()), self._s))
        return elem, chain

    def set_mapping(self, n_lo: int, n_hi: int, lanes_per_chain: int, beads_per_lane: int) -> "Ensemble":
        """Chain-to-wavefront mapping for chains with n_lo <= N <= n_hi."""
        self._chk(lib().ssp_set_mapping(self._h, int(n_lo), int(n_hi), int(lanes_per_chain), int(beads_per_lane)))
        return self

    def set_schedule(self, persistent: bool) -> "Ensemble":
        """Persistent (default) or one-wavefront-per-task schedule of ssp_step."""
        self._chk(lib().ssp_set_schedule(self._h, 1 if persistent else 0))
        return self

    def set_kernel_timing(self, enable: bool) -> "Ensemble":
        self._chk(lib().ssp_set_kernel_timing(self._h, 1 if enable else 0))
        return self

    def kernel_time(self):
        """(ms, launches, bead_steps) of the step kernels timed since the last call."""
        ms, n, bs = ctypes.c_double(), ctypes.c_int64(), ctypes.c_int64()
        self._chk(lib().ssp_kernel_time(self._h, ctypes.byref(ms), ctypes.byref(n), ctypes.byref(bs)))
        return ms.value, n.value, bs.value

    # ------------------------------------------------------- derived views
    def bonds_and_offsets(self):
        """Translation-invariant view: bonds [sumN,3] (R_{i+1}-R_i, NaN at each
        chain's last bead) and anchor offsets d_j = R_{S_j} - A_j [sumN,3] (NaN
        for empty slots), plus S."""
        R, A, S = (x.cpu().numpy() for x in self.state())
        return _invariants(R, A, S, self.N, self.offsets)


def _invariants(R, A, S, N, off):
    bonds = np.full_like(R, np.nan)
    d = np.full_like(R, np.nan)
    for k in range(len(N)):
        o, n = off[k], N[k]
        bonds[o:o + n - 1] = R[o + 1:o + n] - R[o:o + n - 1]
        s = S[o:o + n]
        occ = s >= 0
        d[o:o + n][occ] = R[o + s[occ]] - A[o:o + n][occ]
    return bonds, d, S
