// Plan descriptor: the model compiled into the form the kernels read.
// It lives in device memory; kernels read it with uniform (scalar) loads, so
// coefficient changes never invalidate a captured graph.
//
// Data layout of every spectral array (the "packed half spectrum"):
//   The x transform of a real line has modes kx = 0..Nx/2, with kx = 0 and
//   kx = Nx/2 real.  Column c = 0 stores X(0) + i X(Nx/2); columns
//   c = 1..Nx/2-1 store X(c).  A line therefore holds exactly Nx/2 complex
//   values, and the y (and z) transforms of column 0 give
//   S(0,k) = phi(0,k) + i phi(Nx/2,k), both Hermitian along the other axes.
//   Along the update axis u (y in 2D, z in 3D) a "packed" line (column 0 in
//   2D; column 0 with ky = 0 or Ny/2 in 3D) is kept in slot form: slot u in
//   (0, L/2) holds the kx = 0 mode, slot u in (L/2, L) the kx = Nx/2 mode at
//   index L - u, and slots 0 and L/2 hold the two real self-conjugate modes as
//   (re of kx = 0, re of kx = Nx/2).  Every slot is then one update.
//   Columns are grouped in tiles of TC; arrays are stored
//     2D:  [ctile][y][TC]                      (state, exchanges)
//     3D:  state and z-pass input  [y][ctile][z][TC]
//          y-pass and x-pass arrays [z][ctile][y][TC]
//   so that every kernel reads or writes whole contiguous blocks.
#pragma once

#include <stdint.h>
#include <hip/hip_runtime.h>

#define PSS_MAXF 4    // fields
#define PSS_MAXM 8    // monomials per operator
#define PSS_MAXT 32   // terms
#define PSS_MAXCH 8   // real-space product channels
#define PSS_MAXPT 8   // products per channel
#define PSS_MAXD 8    // Fourier-space (single linear factor) terms
#define PSS_MAXPOW 8  // largest factor power / operator power
#define PSS_MAXI 4    // intermediate (non-dynamic) fields
#define PSS_MAXG 8    // factor slots: distinct fields in real-space products
#define PSS_MAXO 3    // outputs (target field, operator) of one product channel

namespace pss {

struct DevMono {
    float coef;
    int8_t q2, invq, ix, iy, iz, ipow;  // ipow = (ix + iy + iz) mod 4
    int8_t pad[2];
};

// An operator: the pure (q^2)^j monomials folded into dense Horner
// coefficients, plus the monomials with 1/|q| or i q_i factors listed apart.
struct DevOp {
    float poly[PSS_MAXPOW + 1];  // coefficient of (q^2)^j, j = 0..8
    int32_t n;                   // monomials with 1/|q| or i q_i factors
    int32_t deg;                 // highest j with poly[j] != 0 (0 if none)
    DevMono m[PSS_MAXM];
};

struct DevProd {
    float coef;
    int8_t pow[PSS_MAXG];  // power of each factor slot (read as one 64-bit word)
};

// A real-space product channel: F[sum_p coef_p prod_g u_g^pow] is formed once
// and feeds nout field updates, output o adding op[o](q) times it to field
// target[o] (distinct targets; e.g. the stress products of a flow model feed
// every velocity component).
struct DevChannel {
    int32_t nprod;
    int32_t nout;
    int32_t target[PSS_MAXO];
    DevOp op[PSS_MAXO];
    DevProd prod[PSS_MAXPT];
};

struct DevDirect {
    int32_t target, src;  // src: dynamic field, or PSS_MAXF + intermediate
    DevOp op;
};

// An intermediate field (Sec. "Writing models": a field defined by an
// equation without a time derivative), linear in the dynamic fields:
//   psi = sum_k op_k(q) phi_{src_k} / (1 - L_psi(q)),
// L_psi the sum of its implicit operators.  Factor slots and linear terms name
// it as source PSS_MAXF + its index.
struct DevInterm {
    int32_t nsrc;
    int32_t src[PSS_MAXF];  // dynamic field of each linear term
    DevOp op[PSS_MAXF];
    DevOp den;  // L_psi
};

struct DevMask {
    // keep a mode iff  (RADIAL) sum_i w_i k_i^2 * den2 < rhs
    //                  (PER_AXIS) den * |k_i| < num * h_i on every axis
    int64_t w[3];
    int64_t den2, rhs;
    int32_t num, den;
    int32_t h[3];
    int32_t shape;  // 0 radial, 1 per axis, 2 keep all
    int32_t ncol;   // packed columns holding kept modes (c < ncol)
    int32_t ylo;    // 3D: kept |ky| <= ylo (band of the y axis)
    int32_t pad;
};

struct DevPlan {
    int32_t ndim;
    int32_t n[3];      // Nx, Ny, Nz (Nz = 1 in 2D)
    int32_t nf, nch, ng, nd;
    float qs[3];       // 2 pi / (N_i dx_i)
    float dt;
    float inv_n;       // 1 / (Nx Ny Nz)
    float amp_pair;    // sqrt(dt N / dV): sqrt(2 dt/dV) * sqrt(N/2)
    float amp_self;    // sqrt(2 dt N / dV)
    uint32_t key0, key1;
    int32_t noisy[PSS_MAXF];
    int32_t fid[PSS_MAXF];     // declaration index of each dynamic field (its random-number key)
    int32_t gfield[PSS_MAXG];  // factor slot -> dynamic field, or PSS_MAXF + intermediate
    DevMask mask[PSS_MAXG];    // per factor slot
    DevOp implicit_op[PSS_MAXF];
    DevOp noise_op[PSS_MAXF];
    DevDirect direct[PSS_MAXD];
    DevChannel ch[PSS_MAXCH];
    int32_t general;  // some operator has 1/|q| or i q_i monomials (general list), or ni > 0
    int32_t ni;
    DevInterm interm[PSS_MAXI];
    // boundary frames: after every step field f takes value[i] at site[i] of
    // real space (x fastest), i < nframe[f]; entries (site, value bits)
    const int2* frame[PSS_MAXF];
    int32_t nframe[PSS_MAXF];
};

}  // namespace pss
