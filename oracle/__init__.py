"""FP64 CPU oracle for the single-chain slip-spring ensemble.

TEST INFRASTRUCTURE ONLY: only the tests, the package smoke check and the
benchmark's CPU-baseline leg may import this module.  The product path (the
HIP library and its binding) never loads it, and the two share no code.

This module is a thin ctypes wrapper around ``ssp_oracle.c`` (plain C, FP64,
OpenMP over chains); every piece of arithmetic lives in the C file, which
cites the paper section each step follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ssp_oracle.c")
_LIB = os.path.join(_HERE, "libssp_oracle.so")

# Philox counter purposes (step hi | purpose << 24 in the last counter word).
P_INIT_BOND, P_INIT_Z, P_INIT_S, P_INIT_ANCHOR, P_NOISE, P_SLOT, P_ANCHOR, P_NOISE2 = 1, 2, 3, 4, 5, 6, 7, 8

# Event bits reported per slot by a single step.
EV_HOP_UP, EV_HOP_DOWN, EV_DESTROY, EV_CREATE_FIRST, EV_CREATE_LAST = 1, 2, 4, 8, 16


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (-O2, OpenMP, strict IEEE: no -ffast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c99", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        i32p, i64p, f64p, u32p, u8p = P(ctypes.c_int32), P(ctypes.c_int64), P(ctypes.c_double), P(ctypes.c_uint32), P(ctypes.c_uint8)
        L.ssp_oracle_philox.argtypes = [u32p, u32p, u32p]
        L.ssp_oracle_u01.argtypes = [ctypes.c_uint32]
        L.ssp_oracle_u01.restype = ctypes.c_double
        L.ssp_oracle_normals3.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int64, f64p]
        L.ssp_oracle_block.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, ctypes.c_int64, ctypes.c_int64, u32p]
        L.ssp_oracle_step_noise.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int64, ctypes.c_int64, f64p]
        L.ssp_oracle_slot_words.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int64, ctypes.c_int64, u32p]
        L.ssp_oracle_hop_prob.argtypes = [ctypes.c_int, f64p, f64p, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.ssp_oracle_hop_prob.restype = ctypes.c_double
        L.ssp_oracle_init.argtypes = [ctypes.c_int, i32p, i64p, i64p, ctypes.c_double, ctypes.c_double, ctypes.c_uint64, f64p, f64p, i32p]
        L.ssp_oracle_stress.argtypes = [ctypes.c_int, i32p, i64p, ctypes.c_double, f64p, f64p, i32p, f64p]
        L.ssp_oracle_step.argtypes = [ctypes.c_int, i32p, i64p, i64p, f64p, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      ctypes.c_double, ctypes.c_int, ctypes.c_uint64, ctypes.c_int64, f64p, f64p, i32p, u8p, f64p]
        L.ssp_oracle_run.argtypes = [ctypes.c_int, i32p, i64p, i64p, f64p, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, ctypes.c_int, ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, ctypes.c_int64,
                                     f64p, f64p, i32p, f64p]
        L.ssp_oracle_run.restype = ctypes.c_int64
        L.ssp_oracle_multitau.argtypes = [ctypes.c_int64, f64p, f64p, ctypes.c_int, ctypes.c_int, f64p, i64p]
        L.ssp_oracle_threads.argtypes = []
        L.ssp_oracle_threads.restype = ctypes.c_int
        L.ssp_oracle_set_threads.argtypes = [ctypes.c_int]
        L.ssp_oracle_step_forced.argtypes = [ctypes.c_int, i32p, i64p, i64p, f64p, ctypes.c_double, ctypes.c_double,
                                             ctypes.c_uint64, ctypes.c_int64, f64p, f64p, i32p, i32p]
        L.ssp_oracle_adjoint.argtypes = [ctypes.c_int, i32p, i64p, i64p, f64p, ctypes.c_double, ctypes.c_double,
                                         ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, f64p, f64p, i32p,
                                         ctypes.c_int64, ctypes.c_int, ctypes.c_int, f64p, f64p]
        _lib = L
    return _lib


def _p(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def philox(counter, key):
    """Philox4x32-10 block for a 4-word counter and 2-word key."""
    c = np.ascontiguousarray(counter, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().ssp_oracle_philox(_p(c, ctypes.c_uint32), _p(k, ctypes.c_uint32), _p(out, ctypes.c_uint32))
    return out


def set_threads(n: int) -> None:
    """Threads (OpenMP) of the oracle's later calls."""
    lib().ssp_oracle_set_threads(int(n))


def threads() -> int:
    """OpenMP threads the oracle's loops over chains use."""
    return int(lib().ssp_oracle_threads())


def u01(w: int) -> float:
    return lib().ssp_oracle_u01(int(w) & 0xFFFFFFFF)


def block(seed, purpose, index, chain, step):
    out = np.zeros(4, dtype=np.uint32)
    lib().ssp_oracle_block(seed, purpose, index, chain, step, _p(out, ctypes.c_uint32))
    return out


def normals3(seed, purpose, index, chain, step):
    out = np.zeros(3)
    lib().ssp_oracle_normals3(seed, purpose, index, chain, step, _p(out, ctypes.c_double))
    return out


def step_noise(seed, index, chain, step):
    """Noise normals of bead `index` at time step `step` (step-pair layout)."""
    out = np.zeros(3)
    lib().ssp_oracle_step_noise(seed, index, chain, step, _p(out, ctypes.c_double))
    return out


def slot_words(seed, index, chain, step):
    """(hop word, reconstruction word) of slot `index` at time step `step`."""
    out = np.zeros(2, dtype=np.uint32)
    lib().ssp_oracle_slot_words(seed, index, chain, step, _p(out, ctypes.c_uint32))
    return out


def hop_prob(R, a, i, direction, dt=0.01, ns=0.5, zeta_s=0.1):
    R = np.ascontiguousarray(R, dtype=np.float64).reshape(-1, 3)
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(3)
    return lib().ssp_oracle_hop_prob(R.shape[0], _p(R, ctypes.c_double), _p(a, ctypes.c_double), int(i), int(direction), dt, ns, zeta_s)


def multitau(x, y, levels=16, lags=16):
    """Block-averaged multiple-tau correlator of one series pair, by definition."""
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    C = np.zeros((levels, lags))
    cnt = np.zeros((levels, lags), dtype=np.int64)
    lib().ssp_oracle_multitau(x.shape[0], _p(x, ctypes.c_double), _p(y, ctypes.c_double), levels, lags,
                              _p(C, ctypes.c_double), _p(cnt, ctypes.c_int64))
    return C, cnt


class Ensemble:
    """Host-side FP64 state of an ensemble of chains (slot capacity C = N)."""

    def __init__(self, n_beads, chain_ids=None, n0=4.0, ns=0.5, zeta_s=0.1, dt=0.01, seed=1, construct_rule=0):
        """construct_rule: 0 = K = C - Z construction attempts (the GPU rule of
        Sec. 3.2), 1 = K = 1 (the CPU rule of Sec. 3.2)."""
        self.N = np.ascontiguousarray(n_beads, dtype=np.int32)
        self.M = int(self.N.shape[0])
        if np.any(self.N < 2):
            raise ValueError("every chain needs N >= 2 beads")
        self.off = np.zeros(self.M, dtype=np.int64)
        if self.M > 1:
            self.off[1:] = np.cumsum(self.N[:-1], dtype=np.int64)
        self.total = int(self.N.sum())
        self.chain_ids = np.ascontiguousarray(np.arange(self.M) if chain_ids is None else chain_ids, dtype=np.int64)
        self.n0, self.ns, self.zeta_s, self.dt, self.seed = float(n0), float(ns), float(zeta_s), float(dt), int(seed)
        self.construct_rule = int(construct_rule)
        self.R = np.zeros((self.total, 3))
        self.A = np.zeros((self.total, 3))
        self.S = np.full(self.total, -1, dtype=np.int32)
        self.step_index = 0

    def _ptrs(self):
        return (_p(self.N, ctypes.c_int32), _p(self.off, ctypes.c_int64), _p(self.chain_ids, ctypes.c_int64))

    def init(self):
        Np, op, cp = self._ptrs()
        lib().ssp_oracle_init(self.M, Np, op, cp, self.n0, self.ns, self.seed,
                              _p(self.R, ctypes.c_double), _p(self.A, ctypes.c_double), _p(self.S, ctypes.c_int32))
        self.step_index = 0
        return self

    def _kappa(self, kappa):
        k = np.zeros((self.M, 9)) if kappa is None else np.asarray(kappa, dtype=np.float64)
        if k.size == 9:
            k = np.broadcast_to(k.reshape(1, 9), (self.M, 9))
        return np.ascontiguousarray(k.reshape(self.M, 9))

    def step(self, kappa=None, want_events=False):
        """One step; returns (events, margin) per slot when want_events."""
        Np, op, cp = self._ptrs()
        k = self._kappa(kappa)
        ev = np.zeros(self.total, dtype=np.uint8) if want_events else None
        mg = np.zeros(self.total) if want_events else None
        lib().ssp_oracle_step(self.M, Np, op, cp, _p(k, ctypes.c_double), self.dt, self.n0, self.ns, self.zeta_s,
                              self.construct_rule, self.seed, self.step_index, _p(self.R, ctypes.c_double), _p(self.A, ctypes.c_double),
                              _p(self.S, ctypes.c_int32),
                              _p(ev, ctypes.c_uint8) if want_events else None,
                              _p(mg, ctypes.c_double) if want_events else None)
        self.step_index += 1
        return (ev, mg) if want_events else None

    def run(self, n_steps, kappa=None, sample_every=1, keep_samples=True):
        """n_steps steps; returns samples [T][M][12] taken after every step whose
        1-based index is a multiple of sample_every."""
        Np, op, cp = self._ptrs()
        k = self._kappa(kappa)
        T = sum(1 for t in range(self.step_index, self.step_index + n_steps) if (t + 1) % sample_every == 0)
        samples = np.zeros((T, self.M, 12)) if keep_samples else None
        lib().ssp_oracle_run(self.M, Np, op, cp, _p(k, ctypes.c_double), self.dt, self.n0, self.ns, self.zeta_s,
                             self.construct_rule, self.seed, self.step_index, n_steps, sample_every, _p(self.R, ctypes.c_double),
                             _p(self.A, ctypes.c_double), _p(self.S, ctypes.c_int32),
                             _p(samples, ctypes.c_double) if keep_samples else None)
        self.step_index += n_steps
        return samples

    def stress(self):
        out = np.zeros((self.M, 12))
        lib().ssp_oracle_stress(self.M, _p(self.N, ctypes.c_int32), _p(self.off, ctypes.c_int64), self.ns,
                                _p(self.R, ctypes.c_double), _p(self.A, ctypes.c_double), _p(self.S, ctypes.c_int32),
                                _p(out, ctypes.c_double))
        return out

    # ---- frozen-event forward and discrete adjoint -------------------------
    def run_record(self, n_steps, kappa=None):
        """n_steps steps keeping the full trajectory: R, A [(n+1)][tot][3], S [(n+1)][tot]."""
        Rt = np.zeros((n_steps + 1, self.total, 3))
        At = np.zeros((n_steps + 1, self.total, 3))
        St = np.zeros((n_steps + 1, self.total), dtype=np.int32)
        Rt[0], At[0], St[0] = self.R, self.A, self.S
        for t in range(n_steps):
            self.step(kappa)
            Rt[t + 1], At[t + 1], St[t + 1] = self.R, self.A, self.S
        return Rt, At, St

    def step_forced(self, S_next, kappa=None, ns=None):
        """One step with the slot decisions given (S after the step)."""
        Np, op, cp = self._ptrs()
        k = self._kappa(kappa)
        sn = np.ascontiguousarray(S_next, dtype=np.int32)
        lib().ssp_oracle_step_forced(self.M, Np, op, cp, _p(k, ctypes.c_double), self.dt,
                                     self.ns if ns is None else float(ns), self.seed, self.step_index,
                                     _p(self.R, ctypes.c_double), _p(self.A, ctypes.c_double),
                                     _p(self.S, ctypes.c_int32), _p(sn, ctypes.c_int32))
        self.step_index += 1

    def adjoint(self, Rt, At, St, kappa=None, step0=0, comp=3, init_window=True):
        """dJ/dkappa [M][3][3] and dJ/dN_s [M] of J = sigma_comp at the end of the
        recorded window (comp: 0..5 = xx yy zz xy yz zx)."""
        Np, op, cp = self._ptrs()
        k = self._kappa(kappa)
        T = Rt.shape[0] - 1
        Rt = np.ascontiguousarray(Rt, dtype=np.float64)
        At = np.ascontiguousarray(At, dtype=np.float64)
        St = np.ascontiguousarray(St, dtype=np.int32)
        gk = np.zeros((self.M, 9))
        gns = np.zeros(self.M)
        lib().ssp_oracle_adjoint(self.M, Np, op, cp, _p(k, ctypes.c_double), self.dt, self.ns, self.seed, step0, T,
                                 _p(Rt, ctypes.c_double), _p(At, ctypes.c_double), _p(St, ctypes.c_int32),
                                 self.total, comp, 1 if init_window else 0, _p(gk, ctypes.c_double),
                                 _p(gns, ctypes.c_double))
        return gk.reshape(self.M, 3, 3), gns

    # Relative, translation-invariant views used for comparisons.
    def bonds(self):
        out = []
        for k in range(self.M):
            o, n = self.off[k], self.N[k]
            out.append(self.R[o + 1:o + n] - self.R[o:o + n - 1])
        return out

    def anchor_offsets(self):
        """d_j = R_{S_j} - A_j for every slot (NaN for empty slots)."""
        d = np.full((self.total, 3), np.nan)
        for k in range(self.M):
            o, n = self.off[k], self.N[k]
            s = self.S[o:o + n]
            occ = s >= 0
            d[o:o + n][occ] = self.R[o + s[occ]] - self.A[o:o + n][occ]
        return d
