"""torch.autograd binding of the Model B adjoint.

ModelBLoss(n, dt, seed, nsteps, S_target) holds one 2D Model B lattice.
Calling it with the real initial field phi0 (torch, float32, shape (Ny, Nx))
and theta = (a, b, k, D) (torch, 4 values) returns the structure-factor loss
L(phi0, theta) after nsteps steps as a 0-d float64 tensor.

The forward call runs only the forward trajectory.  When an input needs a
gradient it records the checkpoints on the way (pss_adjoint_model_b_forward,
a checkpoint every ckpt_every steps, the noise fixed by its Philox counters);
backward() then runs the reverse sweep (pss_adjoint_model_b_backward) and
writes dL/dphi0 straight into a device tensor.  When no input needs a
gradient the forward is the plain run (pss_step) and the loss comes from the
shell averages of the final spectrum.

One lattice holds one tape: a new forward call on the same ModelBLoss releases
the tape of the previous call, whose backward() then raises.
"""

import numpy as np
import torch

from . import Lattice, Mono, model_b


class _Loss(torch.autograd.Function):
    @staticmethod
    def forward(ctx, phi0, theta, owner):
        want = bool(ctx.needs_input_grad[0] or ctx.needs_input_grad[1])
        loss, tape = owner._forward(phi0, theta, want)
        ctx.tape = tape
        ctx.owner = owner
        ctx.phi_meta = (phi0.shape, phi0.dtype, phi0.device)
        ctx.theta_meta = (theta.dtype, theta.device)
        return torch.tensor(loss, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gout):
        tape = ctx.tape
        if tape is None or ctx.owner._tape is not tape:
            raise RuntimeError("the adjoint tape of this forward call was released by a later call")
        shape, dtype, device = ctx.phi_meta
        if device.type == "cuda":
            gphi = torch.empty(shape, dtype=torch.float32, device=device)
        else:
            gphi = np.empty(shape, dtype=np.float32)
        gtheta = tape.backward(gphi)
        tape.close()
        ctx.owner._tape = None
        if not isinstance(gphi, torch.Tensor):
            gphi = torch.from_numpy(gphi)
        gphi = gphi.to(dtype)
        tdtype, tdevice = ctx.theta_meta
        gtheta = torch.as_tensor(gtheta, dtype=tdtype, device=tdevice)
        g = gout.to(torch.float64)
        return (g * gphi.to(torch.float64)).to(dtype), (g.to(tdevice) * gtheta.to(torch.float64)).to(tdtype), None


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
        self._tape = None

    def __call__(self, phi0, theta):
        return _Loss.apply(phi0, theta, self)

    def _forward(self, phi0, theta, record):
        if self._tape is not None:
            self._tape.close()
            self._tape = None
        a, b, k, D = (float(v) for v in theta.detach().cpu().reshape(-1).tolist())
        t_imp, t_nl = self.terms
        lat = self.lat
        lat.set_coef(t_imp, 0, -a)
        lat.set_coef(t_imp, 1, -k)
        lat.set_coef(t_nl, 0, -b)
        lat.noise(self.field, [Mono(D, q2=1)])
        lat.load(self._start)
        lat.upload(self.field, phi0.detach().contiguous())
        if record:
            loss, tape = lat.adjoint_forward(self.nsteps, self.S_target, self.ckpt_every)
            self._tape = tape
            return loss, tape
        lat.step(self.nsteps)
        S, _ = lat.structure_factor(self.field)
        return float(np.sum((S - self.S_target) ** 2)), None
