"""The two energies of the local Hamiltonian as a differentiable torch function.

Sec. 2.4 and Sec. 5: the minimisation needs the gradient of the energy with
respect to the orbital coefficients.  Both energies are quadratic forms of the
coefficients with symmetric operators,
    E_loc = sum_i f_i <c_i, Hloc c_i>,  Hloc = A M^T V M S,
    E_kin = sum_i f_i <c_i, Kin c_i>,   Kin  = A K S,
(S: synthesis, A = S^T its inverse since the wavelet transform is orthogonal,
M: magic filter, K: the kinetic filter) and E_loc is linear in the potential,
so
    dE_loc/dc_i = 2 f_i Hloc c_i,   dE_kin/dc_i = 2 f_i Kin c_i,
    dE_loc/dV   = rho = sum_i f_i psi_i^2.
The backward pass is therefore one more local H*psi with its two parts
weighted by the incoming gradients and the occupations (wvl_energy_gradient),
run by the library like the forward one; torch only holds the buffers.

Inputs are float64 tensors; a plan of another precision converts them on the
device (the compensated form keeps about 1e-10 of relative accuracy).
"""

import torch

from . import ops


def _to_plan(plan, c64):
    return c64 if plan.prec == "f64" else plan.convert(c64, "f64", plan.prec, plan.elems)


class LocalEnergy(torch.autograd.Function):
    """(E_loc, E_kin) = LocalEnergy.apply(c, V, plan).

    c: packed float64 coefficients of the plan's batch (plan.elems,); V: the
    float64 potential (shared: one grid; otherwise packed per orbital).  The
    gradient with respect to V is available for a shared potential."""

    @staticmethod
    def forward(ctx, c, V, plan):
        if c.dtype != torch.float64 or V.dtype != torch.float64:
            raise TypeError("LocalEnergy takes float64 tensors")
        c = c.contiguous()
        V = V.contiguous()
        r = plan.local_hpsi(_to_plan(plan, c), V, rho=plan.shared_v, energies=True)
        ctx.plan = plan
        ctx.save_for_backward(c, V, r["rho"] if r["rho"] is not None else torch.empty(0))
        e = r["energies"]
        return e[0].clone(), e[1].clone()

    @staticmethod
    def backward(ctx, g_loc, g_kin):
        plan = ctx.plan
        c, V, rho = ctx.saved_tensors
        gl = 0.0 if g_loc is None else float(g_loc)
        gk = 0.0 if g_kin is None else float(g_kin)
        grad_c = grad_V = None
        if ctx.needs_input_grad[0]:
            # 2 f_b (g_loc Hloc + g_kin Kin) c_b, occupations applied by the library
            grad_c = plan.to_f64(plan.energy_gradient(_to_plan(plan, c), V, gl, gk))
        if ctx.needs_input_grad[1]:
            if not plan.shared_v:
                raise NotImplementedError("dE/dV needs a shared potential")
            grad_V = gl * rho
        return grad_c, grad_V, None


def local_energy(c, V, plan):
    """Convenience wrapper: (E_loc, E_kin) with autograd support."""
    return LocalEnergy.apply(c, V, plan)
