"""FP64 CPU oracle for the pseudo-spectral stochastic-PDE time step.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute this package: only the test suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code with the HIP
library (no kernels, headers, tables or helpers) and it never imports it.

What it computes follows the paper (cuPSS, arXiv 2405.02410):

* the field equation dphi = F[phi] dt + sqrt(2D) dW with an operator-valued
  noise strength (Introduction, eq:base; Fourier form eq:base2 and the
  conserved-noise remark D(q) = D q^2);
* terms of the form M(q) * prod_k psi_k^{n_k}, with the operator acting on the
  whole product (Sec. "What cuPSS calculates", eq:basereal and
  eq:nonlin_general);
* pseudo-spectral evaluation of nonlinear terms in real space
  (Sec. "Pseudo-spectral integration", eq:cubicexample);
* de-aliasing by zeroing the modes of each factor beyond 2 pi/((n+1) dx)
  (Sec. "De-aliasing");
* the semi-implicit Euler-Maruyama update eq:timeupdate, with the per-step
  procedure listed right after it;
* Fourier-space Gaussian noise with variance 2 D(q) (eq:noise_eq) drawn from
  a counter-based Philox4x32-10 generator (Salmon et al., SC'11) followed by
  the Box-Muller transform (Box & Muller 1958).

Modules
-------
philox        Philox4x32-10, 23-bit uniforms, Box-Muller.
spectral      lattice wavevectors, transforms, de-aliasing masks, q-operators.
model         model description (fields, terms, noise) and the time step.
observables   mass, structure factor, shell averages, domain length.
adjoint       reverse-mode derivative of a Model B trajectory.

Every function states the passage of the paper it follows.  Readings the paper
leaves open are listed in the module that applies them.
"""


