"""torch.autograd front end of the step adjoint.

KSStepEnergy.apply(vext_q, ctx, psi, lam, occ) runs one augmented-subspace
step with the external potential vext_q (device [n_elems][n_q]) and returns
the step's Kohn-Sham energy E_KS as a 0-d tensor; its backward calls the
hand-written adjoint in the HIP library (ks_step_backward), which recomputes
one adjoint block solve instead of storing CG iterates.  The inputs psi, lam
(the step's starting orbitals and eigenvalues) are held fixed.
"""
import torch


class KSStepEnergy(torch.autograd.Function):
    @staticmethod
    def forward(fctx, vext_q, ks, psi, lam, occ, precision="fp64"):
        ks.set_external(vext_q=vext_q.detach())
        p = psi.detach().clone()
        lam_new, rep = ks.scf_step(p, lam, occ, precision)
        e = ks.step_energy()
        fctx.ks = ks
        fctx.psi_new, fctx.lam_new, fctx.report = p, lam_new, rep
        return vext_q.new_tensor(e["KS"])

    @staticmethod
    def backward(fctx, grad_E):
        g, _, _ = fctx.ks.step_backward(dE=float(grad_E), want_forces=False)
        return g, None, None, None, None, None


def step_energy_and_forces(ks, psi, lam, occ, precision="fp64"):
    """E_KS of one step from (psi, lam) and the nuclear forces -dE_KS/dR."""
    p = psi.detach().clone()
    ks.scf_step(p, lam, occ, precision)
    e = ks.step_energy()
    _, F, _ = ks.step_backward(dE=1.0, want_forces=True)
    return e["KS"], F
