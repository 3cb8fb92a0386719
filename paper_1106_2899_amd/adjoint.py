"""torch.autograd.Function around the library's pathwise adjoint.

FinalStress maps per-element flow rates (and the slip-spring strength N_s)
to the ensemble-mean final stress of each element after a window of steps:

    J_e = (1/M_e) sum_{k in e} sigma_c,k(T),   kappa_e = rate_e * D_e,

with D_e a fixed flow-direction tensor per element (simple shear: D_xy = 1;
uniaxial elongation: diag(1, -1/2, -1/2)).  The forward pass records the
window; the backward pass runs the library's reverse pass and returns
dJ_e/drate_e and dJ_e/dN_s, conditioned on the recorded events and random
normals.  With ckpt_every < window the reverse pass replays each checkpoint
segment; with ckpt_every >= window the forward stores the whole trajectory
(about 13 B per bead-step in FP32) and the reverse pass replays nothing.
N_s is a property of the ensemble: the value passed in must equal it (the
gradient with respect to it is still returned).
"""
from __future__ import annotations

import torch

COMPONENTS = {"xx": 0, "yy": 1, "zz": 2, "xy": 3, "yz": 4, "zx": 5}


class FinalStress(torch.autograd.Function):
    @staticmethod
    def forward(ctx, rates, ns, ensemble, directions, window, ckpt_every, component="xy", init_window=True):
        if abs(float(ns) - ensemble.ns) > 1e-12 * max(1.0, abs(ensemble.ns)):
            raise ValueError("ns must equal the ensemble's slip-spring strength")
        dirs = torch.as_tensor(directions, dtype=torch.float64, device=ensemble.device).reshape(-1, 3, 3)
        if dirs.shape[0] == 1:
            dirs = dirs.expand(ensemble.n_elements, 3, 3)
        r = rates.detach().to(device=ensemble.device, dtype=torch.float64).reshape(-1)
        kappa = (r[:, None, None] * dirs).reshape(ensemble.n_elements, 9).contiguous()
        comp = COMPONENTS[component] if isinstance(component, str) else int(component)
        ensemble.forward_record(window, ckpt_every, kappa)
        J = ensemble.element_stress()[:, comp].contiguous()  # element means (library reduction)
        ctx.ensemble, ctx.dirs, ctx.comp, ctx.init_window = ensemble, dirs, comp, init_window
        ctx.rates_device, ctx.rates_dtype = rates.device, rates.dtype
        ctx.ns_is_tensor = torch.is_tensor(ns)
        return J.to(rates.device)

    @staticmethod
    def backward(ctx, gJ):
        e = ctx.ensemble
        g, _ = e.adjoint_elements(ctx.comp, ctx.init_window)         # [E][10] element means
        # kappa_e = rate_e D_e: dJ_e/drate_e = sum_ab D_e,ab dJ_e/dkappa_e,ab
        dr = (g[:, :9].reshape(-1, 3, 3) * ctx.dirs).sum(dim=(1, 2))
        dn = g[:, 9]
        gJ = gJ.to(device=e.device, dtype=torch.float64)
        grad_rates = (gJ * dr).to(device=ctx.rates_device, dtype=ctx.rates_dtype)
        grad_ns = (gJ * dn).sum().to(device=ctx.rates_device) if ctx.ns_is_tensor else None
        return grad_rates, grad_ns, None, None, None, None, None, None


def final_stress(rates, ns, ensemble, directions, window, ckpt_every, component="xy", init_window=True):
    """J [E] = FinalStress.apply(...) (see the class)."""
    return FinalStress.apply(rates, ns, ensemble, directions, window, ckpt_every, component, init_window)
