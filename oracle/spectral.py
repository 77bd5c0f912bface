"""Lattice, transforms, de-aliasing masks and q-operators (oracle; tests only).

Conventions (readings of the paper, each named here because the paper leaves
it open):

* Transform normalisation.  The paper writes a continuum transform with a
  (2 pi)^(-d/2) prefactor (Sec. "Pseudo-spectral integration" and the
  definition after eq:basefourier) and a discrete series without one
  (Sec. "De-aliasing").  The physics is fixed by the real-space equation
  eq:base, and the convention cancels in the pseudo-spectral product of
  eq:cubicexample.  Here: forward DFT unnormalised, phi_hat(k) =
  sum_x phi(x) exp(-i q.x); inverse carries 1/N.
* Mode indices.  Signed integers in numpy.fft.fftfreq order; the Nyquist
  index N_i/2 is read as -N_i/2.  q_i = 2 pi kt_i / (N_i dx_i).
* Nyquist and odd operators.  i q_i is taken as 0 on the Nyquist plane
  (kt_i = -N_i/2), so an odd derivative of a real field stays real; q^2 keeps
  (pi/dx_i)^2 there.  1/|q| is 0 at q = 0.
* Mask geometry.  The paper derives its rule in 1D and then states it with
  |q| (Sec. "De-aliasing").  RADIAL keeps a mode iff
  sum_i (kt_i / (N_i/2))^2 < f^2 (for equal spacings, |q| < f pi/dx);
  PER_AXIS keeps it iff |kt_i|/(N_i/2) < f on every axis.  Equality is
  zeroed (the paper's "|q| < cutoff" branch keeps strictly-below modes).
* Cutoff fraction.  For a factor whose highest nonlinearity has order n the
  paper zeroes |q| > 2 pi/((n+1) dx), i.e. f = 2/(n+1) of Nyquist.
  TWO_THIRDS uses f = 2/3 for every factor; PAPER_ORDER uses 2/(n+1).
  Mask decisions are taken in exact integer arithmetic.
"""

import math

import numpy as np

try:  # scipy.fft is a library primitive; numpy.fft is the fallback.
    import scipy.fft as _sfft
except Exception:  # pragma: no cover
    _sfft = None

# Dealiasing rules and shapes (same numbering as the C interface; the values
# are a public convention, not shared code).
DEALIAS_TWO_THIRDS = 0
DEALIAS_PAPER_ORDER = 1
DEALIAS_NONE = 2
SHAPE_RADIAL = 0
SHAPE_PER_AXIS = 1

WORKERS = 1  # threads for scipy.fft; the CPU baseline may raise it


def fftn(a):
    """Unnormalised forward DFT over all axes."""
    if _sfft is not None:
        return _sfft.fftn(a, workers=WORKERS)
    return np.fft.fftn(a)


def ifftn(a):
    """Inverse DFT over all axes, with the 1/N factor."""
    if _sfft is not None:
        return _sfft.ifftn(a, workers=WORKERS)
    return np.fft.ifftn(a)


class Lattice:
    """Periodic lattice of shape n = (nz, ny, nx) (array axis order z, y, x).

    `dims` is 1, 2 or 3; unused leading axes have length 1.  The linear site
    or mode index used to key random numbers is L = (z*Ny + y)*Nx + x.
    """

    def __init__(self, nx, ny=1, nz=1, dx=1.0, dy=1.0, dz=1.0):
        self.nx, self.ny, self.nz = int(nx), int(ny), int(nz)
        self.dx, self.dy, self.dz = float(dx), float(dy), float(dz)
        self.shape = (self.nz, self.ny, self.nx)
        self.N = self.nx * self.ny * self.nz
        self.dV = self.dx * self.dy * self.dz
        # signed mode indices, Nyquist read as -N/2
        self.kt = [self._signed(n) for n in (self.nx, self.ny, self.nz)]
        kx = self.kt[0][None, None, :]
        ky = self.kt[1][None, :, None]
        kz = self.kt[2][:, None, None]
        self.k_int = (kx, ky, kz)
        self.q = [2 * np.pi * kx / (self.nx * self.dx),
                  2 * np.pi * ky / (self.ny * self.dy),
                  2 * np.pi * kz / (self.nz * self.dz)]
        self.q2 = self.q[0] ** 2 + self.q[1] ** 2 + self.q[2] ** 2
        self.q2 = np.broadcast_to(self.q2, self.shape).copy()
        self.qabs = np.sqrt(self.q2)
        # i*q_i with the Nyquist plane set to zero
        self.iq = []
        for i, n in enumerate((self.nx, self.ny, self.nz)):
            qi = self.q[i].copy()
            if n % 2 == 0:
                qi = np.where(self.k_int[i] == -(n // 2), 0.0, qi)
            self.iq.append(np.broadcast_to(1j * qi, self.shape))
        # linear index of each mode and of its negative
        z = np.arange(self.nz)[:, None, None]
        y = np.arange(self.ny)[None, :, None]
        x = np.arange(self.nx)[None, None, :]
        self.lin = ((z * self.ny + y) * self.nx + x).astype(np.int64)
        xm = (-x) % self.nx
        ym = (-y) % self.ny
        zm = (-z) % self.nz
        self.lin_neg = ((zm * self.ny + ym) * self.nx + xm).astype(np.int64)
        self.lin = np.broadcast_to(self.lin, self.shape)
        self.lin_neg = np.broadcast_to(self.lin_neg, self.shape)

    @staticmethod
    def _signed(n):
        k = np.arange(n)
        k = np.where(k >= (n + 1) // 2, k - n, k)  # fftfreq order
        if n % 2 == 0:
            k = np.where(k == n // 2, -(n // 2), k)
        return k.astype(np.int64)

    # -- de-aliasing (Sec. "De-aliasing") --------------------------------
    def mask(self, num, den, shape=SHAPE_RADIAL):
        """Keep-mask for cutoff fraction f = num/den of the Nyquist index.

        Integer form of sum_i (kt_i/(N_i/2))^2 < f^2 (RADIAL) or of
        |kt_i|/(N_i/2) < f on each axis (PER_AXIS).  Axes of length 1 only
        hold kt = 0 and are skipped.
        """
        halves = []
        ks = []
        for i, n in enumerate((self.nx, self.ny, self.nz)):
            if n == 1:
                continue
            halves.append(n // 2)
            ks.append(self.k_int[i])
        if not halves:
            return np.ones(self.shape, dtype=bool)
        if shape == SHAPE_PER_AXIS:
            keep = np.ones(self.shape, dtype=bool)
            for k, h in zip(ks, halves):
                keep &= (den * np.abs(k)) < (num * h)
            return keep
        # exact integer form: multiply through by l = lcm_i(h_i^2)
        l = 1
        for h in halves:
            l = math.lcm(l, h * h)
        lhs = 0
        for k, h in zip(ks, halves):
            lhs = lhs + (k * k) * (l // (h * h))
        lhs = np.broadcast_to(lhs, self.shape).astype(np.int64)
        return (lhs * (den * den)) < (num * num * l)

    # -- operators (Sec. "Reserved keywords", "Adding noise") -----------
    def operator(self, monos):
        """Complex value of sum_m coef_m (q^2)^a_m |q|^-b_m (iqx)^cx (iqy)^cy (iqz)^cz."""
        out = np.zeros(self.shape, dtype=np.complex128)
        for m in monos:
            v = np.full(self.shape, complex(m.coef), dtype=np.complex128)
            if m.q2:
                v = v * self.q2 ** m.q2
            if m.invq:
                with np.errstate(divide="ignore"):
                    inv = np.where(self.qabs > 0, 1.0 / np.where(self.qabs > 0, self.qabs, 1.0), 0.0)
                v = v * inv ** m.invq
            for i, p in enumerate(m.iq):
                if p:
                    v = v * self.iq[i] ** p
            out += v
        return out


class Mono:
    """One operator monomial coef * (q^2)^q2 * |q|^(-invq) * prod_i (i q_i)^iq[i]."""

    def __init__(self, coef, q2=0, invq=0, iq=(0, 0, 0)):
        self.coef = float(coef)
        self.q2 = int(q2)
        self.invq = int(invq)
        self.iq = tuple(int(v) for v in iq) + (0,) * (3 - len(iq))

    def __repr__(self):
        return f"Mono({self.coef}, q2={self.q2}, invq={self.invq}, iq={self.iq})"
