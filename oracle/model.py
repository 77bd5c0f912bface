"""Model description and the semi-implicit stochastic time step (oracle; tests only).

A model is a set of real fields phi_f on a periodic lattice, each obeying
(Sec. "What cuPSS calculates", eq:basereal and eq:basefourier)

    d/dt phi_f = L_f(q) phi_f + sum_t M_t(q) F[ prod_k u_{g_k}^{p_k} ] + noise_f

where L_f is the implicit self-linear operator, each explicit term t has an
operator M_t acting on the whole product (the paragraph on explicit terms in
Sec. "Writing models"), and the noise has Fourier variance 2 D_f(q)
(eq:noise_eq; Sec. "Adding noise").

One step from phi^n to phi^{n+1} follows the six-step list after
eq:timeupdate:

1. compute every intermediate (non-dynamic) field from the step-n state, in
   the order the fields were declared (Sec. "Writing models");
2. de-alias each factor field according to the highest-order term it enters
   (Sec. "De-aliasing");
3. transform the de-aliased factors to real space and multiply;
4. transform each product back to Fourier space;
5. draw Fourier-space Gaussian noise for every noisy field and scale it;
6. advance every dynamic field with eq:timeupdate,
       phi^{n+1} = (phi^n + dt sum_t M_t N_t + sqrt(dt) eta) / (1 - dt L(q)).

Readings of points the paper leaves open:

* Sign convention of terms: every term, implicit or explicit, is written on
  the right-hand side of d/dt phi (eq:basereal).  The equation-string form
  "dt phi + lhs = rhs" of Sec. "Writing models" maps to implicit operators
  equal to minus the lhs prefactor.
* An explicit term with a single factor of power 1 is linear; it needs neither
  de-aliasing nor a real-space round trip, so its Fourier value is the
  factor's own spectrum (the round trip is the identity).
* Intermediate fields.  A field without a time derivative is defined by the
  equation "psi + lhs = rhs" of Sec. "Writing models": its implicit terms
  (linear in psi, written on the right-hand side like those of a dynamic
  field, so L_psi is minus the lhs prefactor) and its explicit terms give
      psi_hat = sum_t M_t N_t / (1 - L_psi(q)),
  the same form as eq:timeupdate without a previous value, time step or
  noise.  The paper's example psi + psi q^2 = -q^2 phi has L_psi = -q^2 and
  gives psi_hat = -q^2 (1 + q^2)^-1 phi_hat.  An intermediate may use the
  dynamic fields and the intermediates declared before it; it is evaluated
  from the step-n state, so it enters the step like any explicit term.
* Multi-field update order: all explicit terms are evaluated from the step-n
  state, then every field is advanced (Jacobi), as the list orders
  "calculate each N_ij" before "advance each field".
* Noise normalisation (eq:noise_eq uses continuum delta functions): lattice
  white noise with <xi_x xi_x'> = delta_xx'/dV, so the Fourier amplitude of the
  increment is sigma(q) xi_hat(k) with sigma = sqrt(2 D(q) dt / dV) and
  <|xi_hat|^2> = N; the sqrt(dt) of eq:timeupdate is inside sigma.
* Real fields: xi_hat is Hermitian.  A mode k and its partner -k share one
  Philox draw, keyed by the smaller of their linear indices c(k); the owner
  (linear index == c) takes sqrt(N/2)(g1 + i g2), the partner its conjugate,
  and a self-conjugate mode takes sqrt(N) g1.  The Philox counter is
  (c(k), step, field, 0) with the 64-bit seed as key.
* Real space is the real part of the inverse transform.
* Boundary frames (Sec. "Callback functions": a field is held at fixed
  values on a band of sites by setting its real-space values at the end of
  every step).  Read as: after the update of a step, the field's real space
  (the real part of its inverse transform) takes the frame values on the
  frame sites and the field is transformed back; the next step starts from
  that state.
* Initial fields "uniform in [lo, hi)" take u0 of Philox counter
  (site, 0, field, 1) and set phi = float32(lo + (hi - lo) u0), i.e. the FP64
  value rounded once to binary32, so FP32 and FP64 runs start identically.
"""

import numpy as np

from . import philox
from .spectral import (Lattice, Mono, fftn, ifftn, DEALIAS_TWO_THIRDS,
                       DEALIAS_PAPER_ORDER, DEALIAS_NONE, SHAPE_RADIAL)


class Term:
    def __init__(self, target, implicit, op, factors):
        self.target = int(target)
        self.implicit = bool(implicit)
        self.op = [m if isinstance(m, Mono) else Mono(*m) for m in op]
        self.factors = [(int(g), int(p)) for g, p in factors]

    @property
    def order(self):
        return sum(p for _, p in self.factors)

    @property
    def is_direct(self):
        """Single factor to the first power: applied directly in Fourier space."""
        return len(self.factors) == 1 and self.factors[0][1] == 1


class Model:
    """Fields, terms and noise on a lattice; state kept as full complex spectra."""

    def __init__(self, lattice, dt, seed=0, dealias=DEALIAS_TWO_THIRDS,
                 shape=SHAPE_RADIAL):
        self.lat = lattice
        self.dt = float(dt)
        self.seed = int(seed)
        self.dealias = dealias
        self.mask_shape = shape
        self.names = []
        self.dynamic = []
        self.terms = []
        self.noise = {}
        self.state = []
        self.frames = {}
        self.step_index = 0
        self._cache = None

    # -- construction ---------------------------------------------------
    def add_field(self, name, dynamic=True):
        """A dynamic field (state kept) or an intermediate one (dynamic=False,
        recomputed from the state whenever it is needed)."""
        self.names.append(name)
        self.dynamic.append(bool(dynamic))
        self.state.append(np.zeros(self.lat.shape, dtype=np.complex128) if dynamic else None)
        self._cache = None
        return len(self.names) - 1

    def add_term(self, target, op, factors, implicit=False):
        t = Term(target, implicit, op, factors)
        if implicit and not (t.factors == [(t.target, 1)]):
            raise ValueError("an implicit term must be linear in its own field")
        self.terms.append(t)
        self._cache = None
        return len(self.terms) - 1

    def set_frame(self, field, sites, values):
        """Hold `field` at `values` on the linear site indices `sites` after
        every step (a boundary frame)."""
        if not self.dynamic[int(field)]:
            raise ValueError("an intermediate field has no frame")
        sites = np.asarray(sites, dtype=np.int64).reshape(-1)
        values = np.asarray(values, dtype=np.float64).reshape(-1)
        if sites.shape != values.shape or np.any(sites < 0) or np.any(sites >= self.lat.N):
            raise ValueError("frame sites and values must match and lie on the lattice")
        self.frames[int(field)] = (sites, values)

    def _apply_frames(self):
        for f, (sites, values) in self.frames.items():
            x = ifftn(self.state[f]).real.reshape(-1)
            x[sites] = values
            self.state[f] = fftn(x.reshape(self.lat.shape).astype(np.complex128))

    def set_noise(self, field, op):
        if not self.dynamic[int(field)]:
            raise ValueError("an intermediate field has no noise")
        self.noise[int(field)] = [m if isinstance(m, Mono) else Mono(*m) for m in op]
        self._cache = None

    # -- state ----------------------------------------------------------
    def set_real(self, field, values):
        if not self.dynamic[field]:
            raise ValueError("an intermediate field is defined by its equation")
        values = np.asarray(values, dtype=np.float64).reshape(self.lat.shape)
        self.state[field] = fftn(values.astype(np.complex128))

    def init_uniform(self, field, lo, hi):
        """phi_0 = float32(lo + (hi - lo) u0) at every site (see module notes)."""
        u0 = philox.uniform_site(self.lat.lin, field, self.seed)
        vals = (lo + (hi - lo) * u0).astype(np.float32).astype(np.float64)
        self.set_real(field, vals)
        return vals

    def real(self, field):
        return ifftn(self.spectra()[field]).real

    def spectra(self):
        """Fourier values of every field at the current step: the state of
        each dynamic field, and each intermediate field computed in declaration
        order (step 1 of the list)."""
        c = self._prepare()
        spec = list(self.state)
        for f, dyn in enumerate(self.dynamic):
            if dyn:
                continue
            acc = np.zeros(self.lat.shape, dtype=np.complex128)
            for i, t in enumerate(self.terms):
                if t.target == f and not t.implicit:
                    acc = acc + c["ops"][i] * self._term_hat(t, spec)
            spec[f] = acc / c["denom"][f]
        return spec

    # -- per-plan quantities (computed once, like a plan) ----------------
    def _prepare(self):
        if self._cache is not None:
            return self._cache
        lat = self.lat
        nf = len(self.names)
        lam = [np.zeros(lat.shape, dtype=np.complex128) for _ in range(nf)]
        for t in self.terms:
            if t.implicit:
                lam[t.target] = lam[t.target] + lat.operator(t.op)
        # dynamic: 1 - dt L (eq:timeupdate); intermediate: 1 - L_psi
        denom = [1.0 - (self.dt if self.dynamic[f] else 1.0) * lam[f] for f in range(nf)]
        for f in range(nf):
            if self.dynamic[f]:
                continue
            if np.any(denom[f] == 0):
                raise ValueError("the equation of intermediate field %d is singular at some mode" % f)
            for t in self.terms:
                if t.target == f and not t.implicit:
                    for g, _ in t.factors:
                        if not self.dynamic[g] and g >= f:
                            raise ValueError("an intermediate field may use only intermediates declared before it")
        for f in self.noise:
            if not self.dynamic[f]:
                raise ValueError("an intermediate field has no noise")
        ops = [lat.operator(t.op) for t in self.terms]
        # highest order among the nonlinear terms that contain each field
        order = [0] * nf
        for t in self.terms:
            if t.implicit or t.is_direct:
                continue
            for g, _ in t.factors:
                order[g] = max(order[g], t.order)
        masks = []
        for g in range(nf):
            if order[g] == 0 or self.dealias == DEALIAS_NONE:
                masks.append(None)
            elif self.dealias == DEALIAS_TWO_THIRDS:
                masks.append(lat.mask(2, 3, self.mask_shape))
            elif self.dealias == DEALIAS_PAPER_ORDER:
                masks.append(lat.mask(2, order[g] + 1, self.mask_shape))
            else:
                raise ValueError("unknown dealias rule")
        sigma = {}
        for f, op in self.noise.items():
            D = lat.operator(op)
            if np.any(np.abs(D.imag) > 0) or np.any(D.real < 0):
                raise ValueError("noise operator must be real and non-negative")
            sigma[f] = np.sqrt(2.0 * D.real * self.dt / lat.dV)
        self._cache = dict(denom=denom, ops=ops, masks=masks, sigma=sigma)
        return self._cache

    # -- noise (step 5) ---------------------------------------------------
    def noise_hat(self, field, step):
        """Unit-variance Hermitian white noise xi_hat(k) for (step, field)."""
        lat = self.lat
        c = np.minimum(lat.lin, lat.lin_neg)
        g1, g2 = philox.gaussian_pair(c, step, field, self.seed)
        own = lat.lin == c
        selfc = lat.lin == lat.lin_neg
        half = np.sqrt(lat.N / 2.0)
        xi = np.where(own, half * (g1 + 1j * g2), half * (g1 - 1j * g2))
        xi = np.where(selfc, np.sqrt(float(lat.N)) * g1 + 0j, xi)
        return xi

    # -- one step ----------------------------------------------------------
    def _term_hat(self, t, spec):
        """Fourier transform of term t's product of de-aliased factors (steps
        2-4), the factors' Fourier values taken from `spec`."""
        c = self._prepare()
        if t.is_direct:
            return spec[t.factors[0][0]]
        prod = np.ones(self.lat.shape, dtype=np.float64)
        for g, p in t.factors:
            sg = spec[g]
            if c["masks"][g] is not None:
                sg = sg * c["masks"][g]
            u = ifftn(sg).real
            prod = prod * u ** p
        return fftn(prod.astype(np.complex128))

    def nonlinear_hat(self, t_index):
        """Fourier transform of term t's product of de-aliased factors at the
        current step."""
        return self._term_hat(self.terms[t_index], self.spectra())

    def step(self, nsteps=1):
        c = self._prepare()
        for _ in range(int(nsteps)):
            n = self.step_index
            spec = self.spectra()
            rhs = [np.zeros(self.lat.shape, dtype=np.complex128) for _ in self.names]
            for i, t in enumerate(self.terms):
                if t.implicit or not self.dynamic[t.target]:
                    continue
                rhs[t.target] += c["ops"][i] * self._term_hat(t, spec)
            new = []
            for f in range(len(self.names)):
                if not self.dynamic[f]:
                    new.append(None)
                    continue
                acc = self.state[f] + self.dt * rhs[f]
                if f in c["sigma"]:
                    acc = acc + c["sigma"][f] * self.noise_hat(f, n)
                new.append(acc / c["denom"][f])
            self.state = new
            self._apply_frames()
            self.step_index += 1

    # -- convenience ------------------------------------------------------
    def copy(self):
        m = Model(self.lat, self.dt, self.seed, self.dealias, self.mask_shape)
        m.names = list(self.names)
        m.dynamic = list(self.dynamic)
        m.terms = list(self.terms)
        m.noise = dict(self.noise)
        m.frames = dict(self.frames)
        m.state = [None if s is None else s.copy() for s in self.state]
        m.step_index = self.step_index
        return m


def model_b(lattice, dt, a=-1.0, b=1.0, k=1.0, D=0.01, seed=1,
            dealias=DEALIAS_TWO_THIRDS, shape=SHAPE_RADIAL):
    """Model B (Cahn-Hilliard with conserved noise), Sec. "Example":
    d/dt phi_hat = -q^2 (a + k q^2) phi_hat - b q^2 F[u^3] + conserved noise D q^2.
    """
    m = Model(lattice, dt, seed=seed, dealias=dealias, shape=shape)
    f = m.add_field("phi")
    m.add_term(f, [Mono(-a, q2=1), Mono(-k, q2=2)], [(f, 1)], implicit=True)
    m.add_term(f, [Mono(-b, q2=1)], [(f, 3)])
    if D:
        m.set_noise(f, [Mono(D, q2=1)])
    return m


def two_field_3d(lattice, dt, a=-1.0, b=1.0, k=1.0, c=-0.5, g=0.3, D=0.005,
                 seed=1, dealias=DEALIAS_TWO_THIRDS, shape=SHAPE_RADIAL):
    """Model B field phi coupled to a Model A field psi.

    d/dt phi = lap(a phi + b phi^3 - k lap phi + (g/2) phi psi^2) + conserved noise D q^2
    d/dt psi = -(c psi + psi^3 - lap psi) - g phi psi + noise D
    (the literal coupling reading: (g/2) phi psi^2 inside phi's chemical
    potential and -g phi psi in psi's equation; no single free energy gives both).
    """
    m = Model(lattice, dt, seed=seed, dealias=dealias, shape=shape)
    phi = m.add_field("phi")
    psi = m.add_field("psi")
    m.add_term(phi, [Mono(-a, q2=1), Mono(-k, q2=2)], [(phi, 1)], implicit=True)
    m.add_term(phi, [Mono(-b, q2=1)], [(phi, 3)])
    m.add_term(phi, [Mono(-0.5 * g, q2=1)], [(phi, 1), (psi, 2)])
    m.add_term(psi, [Mono(-c), Mono(-1.0, q2=1)], [(psi, 1)], implicit=True)
    m.add_term(psi, [Mono(-1.0)], [(psi, 3)])
    m.add_term(psi, [Mono(-g)], [(phi, 1), (psi, 1)])
    if D:
        m.set_noise(phi, [Mono(D, q2=1)])
        m.set_noise(psi, [Mono(D)])
    return m


def kpz(lattice, dt, sigma=1.0, lam=1.0, D=0.01, seed=1, dealias=DEALIAS_TWO_THIRDS,
        shape=SHAPE_RADIAL):
    """KPZ interface growth (Sec. "What cuPSS calculates"):
    d/dt phi = sigma lap phi + lam (grad phi)^2 + sqrt(2 D) eta.

    The nonlinearity acts on gradients, not on phi, so it is written with one
    intermediate field per lattice axis, g_i = d_i phi (i q_i phi_hat), and
    the explicit terms lam g_i^2 (Sec. "Writing models").  Noise is not
    conserved, D(q) = D.
    """
    m = Model(lattice, dt, seed=seed, dealias=dealias, shape=shape)
    phi = m.add_field("phi")
    m.add_term(phi, [Mono(-sigma, q2=1)], [(phi, 1)], implicit=True)
    for i, n in enumerate((lattice.nx, lattice.ny, lattice.nz)):
        if n == 1:
            continue
        iq = [0, 0, 0]
        iq[i] = 1
        g = m.add_field("d%s_phi" % "xyz"[i], dynamic=False)
        m.add_term(g, [Mono(1.0, iq=iq)], [(phi, 1)])
        m.add_term(phi, [Mono(lam)], [(g, 2)])
    if D:
        m.set_noise(phi, [Mono(D)])
    return m


def model_h_force_ops(k, ndim=2):
    """Operators of the projected Korteweg force of model_h, per velocity
    component and stress product: {(component, (i, j)): [Mono, ...]} for the
    products g_i g_j, i <= j (g = grad phi), in 2 or 3 dimensions.

    The force -k d_j(g_i g_j) is projected with P_ci = delta_ci + (iq_c)(iq_i)/q^2
    (the Fourier form of the pressure's Poisson equation), so component c
    receives -k sum_ij P_ci (i q_j) F[g_i g_j]; g_i g_j with i != j stands for
    the pairs (i, j) and (j, i).
    """
    ops = {}
    for c in range(ndim):
        for i in range(ndim):
            for j in range(i, ndim):
                monos = []
                pairs = [(i, j)] if i == j else [(i, j), (j, i)]
                for a, bb in pairs:
                    # delta_ca (i q_b)
                    if a == c:
                        iq = [0, 0, 0]
                        iq[bb] += 1
                        monos.append(Mono(-k, iq=iq))
                    # (i q_c)(i q_a)(i q_b) / q^2
                    iq = [0, 0, 0]
                    iq[c] += 1
                    iq[a] += 1
                    iq[bb] += 1
                    monos.append(Mono(-k, invq=2, iq=iq))
                ops[(c, (i, j))] = monos
    return ops


def model_h(lattice, dt, a=-1.0, b=1.0, k=1.0, M=1.0, eta=1.0, D=0.0, seed=1,
            dealias=DEALIAS_TWO_THIRDS, shape=SHAPE_RADIAL):
    """Model H in 2D or 3D (the paper's second benchmark, Sec. "Benchmarking";
    Hohenberg and Halperin's model H): a conserved order parameter advected by
    an incompressible Stokes flow that its interfaces drive,

        d/dt phi = -v . grad phi + M lap mu,      mu = a phi + b phi^3 - k lap phi,
        d/dt v   = eta lap v - grad p - phi grad mu,      div v = 0,

    with conserved noise D q^2 on phi (the flow is deterministic).

    Written in the form this library takes (fields, implicit operators,
    operator-times-product terms):
    * the pressure solves lap p = div f; in Fourier space that is the
      projection f_hat -> P(q) f_hat, P_ij = delta_ij - q_i q_j / q^2,
      which is linear in f and becomes part of each term's operator;
    * -phi grad mu differs from -k d_j(g_i g_j), g = grad phi, by a
      gradient, which P removes, so the force terms are the stress products
      g_i g_j (i <= j) with the operators of model_h_force_ops;
    * g_i are intermediate fields (i q_i phi_hat);
    * advection -v . grad phi = -sum_i v_i g_i (equal to -div(v phi) for a
      solenoidal v).
    Readings: the convective term (v . grad) v is left out (the viscous,
    low-Reynolds form of model H), and the velocity has no noise (per-field
    noise cannot be projected).  Fields: phi, the velocity components (dynamic)
    and the gradient components (intermediate), in that order.
    """
    ndim = 3 if lattice.nz != 1 else 2
    m = Model(lattice, dt, seed=seed, dealias=dealias, shape=shape)
    phi = m.add_field("phi")
    v = [m.add_field("v" + "xyz"[i]) for i in range(ndim)]
    g = [m.add_field("d%s_phi" % "xyz"[i], dynamic=False) for i in range(ndim)]
    for i in range(ndim):
        iq = [0, 0, 0]
        iq[i] = 1
        m.add_term(g[i], [Mono(1.0, iq=iq)], [(phi, 1)])
    # order parameter: M lap mu, advection
    m.add_term(phi, [Mono(-M * a, q2=1), Mono(-M * k, q2=2)], [(phi, 1)], implicit=True)
    m.add_term(phi, [Mono(-M * b, q2=1)], [(phi, 3)])
    for i in range(ndim):
        m.add_term(phi, [Mono(-1.0)], [(v[i], 1), (g[i], 1)])
    # flow: viscosity, projected stress
    ops = model_h_force_ops(k, ndim)
    for c in range(ndim):
        m.add_term(v[c], [Mono(-eta, q2=1)], [(v[c], 1)], implicit=True)
        for i in range(ndim):
            for j in range(i, ndim):
                fac = [(g[i], 2)] if i == j else [(g[i], 1), (g[j], 1)]
                m.add_term(v[c], ops[(c, (i, j))], fac)
    if D:
        m.set_noise(phi, [Mono(D, q2=1)])
    return m
