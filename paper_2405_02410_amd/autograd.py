"""torch.autograd binding of the Model B adjoint (pss_adjoint_model_b).

ModelBLoss(n, dt, seed, nsteps, S_target) holds one 2D Model B lattice.
Calling it with the real initial field phi0 (torch, float32, shape (Ny, Nx))
and theta = (a, b, k, D) (torch, 4 values) returns the structure-factor loss
L(phi0, theta) after nsteps steps as a 0-d tensor whose backward() gives
dL/dphi0 and dL/dtheta.  The forward call already runs the reverse sweep of
the library (checkpointed, with the noise fixed by its Philox counters), so
backward() only scales the stored gradients by the incoming gradient.
"""

import numpy as np
import torch

from . import Lattice, Mono, model_b


class _Loss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi0, theta, owner):
        loss, gtheta, gphi = owner._run(phi0, theta)
        ctx.save_for_backward(torch.from_numpy(gphi).to(phi0.device, phi0.dtype),
                              torch.from_numpy(gtheta).to(theta.device, theta.dtype))
        return torch.tensor(loss, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gout):
        gphi, gtheta = ctx.saved_tensors
        return gout.to(gphi.dtype) * gphi, gout.to(gtheta.dtype) * gtheta, None


class ModelBLoss:
    """L = sum_j (S_j(phi_T) - S_target_j)^2 over shells j >= 1 of a 2D Model B
    run of nsteps from phi0 at step 0, differentiable in phi0 and (a, b, k, D).
    The lattice is built with noise (D q^2), so theta's D may be any value >= 0."""

    def __init__(self, n, dt, seed, nsteps, S_target, ckpt_every=45, dx=None):
        self.lat = Lattice(n, dx=dx, dt=dt, seed=seed)
        self.field, self.terms = model_b(self.lat, D=1.0)
        self.lat.init_uniform(self.field)  # builds the plan; the state is replaced per call
        self._start = self.lat.save()      # step 0
        self.nsteps = int(nsteps)
        self.ckpt_every = int(ckpt_every)
        self.S_target = np.ascontiguousarray(S_target, dtype=np.float64)

    def __call__(self, phi0, theta):
        return _Loss.apply(phi0, theta, self)

    def _run(self, phi0, theta):
        a, b, k, D = (float(v) for v in theta.detach().cpu().reshape(-1).tolist())
        t_imp, t_nl = self.terms
        lat = self.lat
        lat.set_coef(t_imp, 0, -a)
        lat.set_coef(t_imp, 1, -k)
        lat.set_coef(t_nl, 0, -b)
        lat.noise(self.field, [Mono(D, q2=1)])
        lat.load(self._start)
        lat.upload(self.field, phi0.detach().contiguous())
        return lat.adjoint_model_b(self.nsteps, self.S_target, self.ckpt_every)
