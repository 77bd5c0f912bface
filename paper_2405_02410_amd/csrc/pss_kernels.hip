// HIP kernels of the pseudo-spectral stochastic step for gfx950.
//
// One 2D step (eq:timeupdate and the six-step list after it) is two kernels:
//
//   update kernel (lines along y, one or more packed columns per block)
//     forward y-FFT of every product channel  -> N_hat(kx, ky)       (step 4)
//     Philox4x32-10 + Box-Muller noise per mode, in registers        (step 5)
//     phi <- (phi + dt sum M N_hat + sigma xi) / (1 - dt L)          (step 6)
//     de-alias mask, inverse y-FFT of every factor field  -> V       (steps 2-3)
//   x kernel (lines along x, RB rows per block, two real rows per complex FFT)
//     inverse x-FFT of V (C2R) -> u(x, y); products sum c prod u^p   (step 3)
//     forward x-FFT (R2C) -> channel arrays for the next step        (step 4)
//
// The spectral arrays use the packed half-spectrum layout described in
// pss_plan.h: column 0 holds X(kx=0) + i X(kx=Nx/2).  Line transforms are the
// register/LDS transforms of pss_fft.h: a forward transform takes its input in
// digit-reversed order and returns natural order (dit), an inverse transform
// takes natural order and returns digit-reversed order (dif), so every
// per-mode computation sees natural mode order.  A line is held by
// consecutive threads.
//
// Position order.  The arrays that pass between the kernels of a step (the
// de-aliased factors V and the product channels N, and their adjoint
// counterparts) hold, along the update axis, position p = t + m*T the value
// of the digit-reversed index D(t) + m*T.  The update kernel then reads and
// writes them contiguously, and the x kernel (and the 3D y pass), whose work
// does not depend on the coordinate along that axis, simply treat positions
// as rows.  The state and the arrays of the transform modes (uploads,
// downloads) stay in natural order; those gather or scatter at D(t) + m*T.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "pss_device.h"
#include "pss_fft.h"
#include "pss_kernels.h"
#include "pss_plan.h"

namespace pss {

// ----------------------------------------------------------------- twiddles
// Copy of the twiddle table into LDS, in two halves so that the caller can
// issue its own loads in between: every thread loads its (at most P) entries
// at once, then stores them.  The blocks hold at least L/P threads, so P
// entries per thread cover the table.  The caller puts a block barrier
// between the store and the first transform.
template <int L, int P>
__device__ __forceinline__ void load_twiddles(float2 (&w)[P], const float2* __restrict__ src, int tid, int nthr) {
    // unconditional loads (the index wraps, L is a power of two) keep the
    // memory counter exact for the loads the caller issues next
#pragma unroll
    for (int k = 0; k < P; ++k) w[k] = src[(tid + k * nthr) & (L - 1)];
}
template <int L, int P>
__device__ __forceinline__ const float2* store_twiddles(float2* dst, const float2 (&w)[P], int tid, int nthr) {
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const int i = tid + k * nthr;
        if (i < L) dst[i] = w[k];
    }
    return dst;
}

// Sum of NV per-thread FP64 values over the block in a fixed order (a
// shuffle tree inside each wave, then the waves in index order), added by
// thread 0 into this block's own slot[0..NV).  Launches with the same grid
// add into the same slots in stream order, so the slots, and a fixed-order
// sum over them, do not depend on how the blocks are scheduled.  Every thread
// of the block calls it; the block is whole waves or a part of one.
template <int NV>
__device__ __forceinline__ void block_sum_to_slot(double (&v)[NV], double* __restrict__ slot) {
    __shared__ double red[64 * NV];
    const int nt = blockDim.x, tid = threadIdx.x;
    const bool waves = (nt & 63) == 0;
    if (waves) {
#pragma unroll
        for (int i = 0; i < NV; ++i)
#pragma unroll
            for (int o = 32; o > 0; o >>= 1) v[i] += __shfl_xor(v[i], o, 64);
        if ((tid & 63) == 0)
#pragma unroll
            for (int i = 0; i < NV; ++i) red[(tid >> 6) * NV + i] = v[i];
    } else {
#pragma unroll
        for (int i = 0; i < NV; ++i) red[tid * NV + i] = v[i];
    }
    __syncthreads();
    if (tid == 0) {
        const int n = waves ? nt >> 6 : nt;
#pragma unroll
        for (int i = 0; i < NV; ++i) {
            double acc = 0.0;
            for (int w = 0; w < n; ++w) acc += red[w * NV + i];
            slot[i] += acc;
        }
    }
}

// ----------------------------------------------------------------- modes
struct ModeQ {
    float q2;
    float invq;  // 1/|q| (0 at q = 0)
    float iq[3];
};

// signed index of mode i on an axis of even length n (Nyquist read as -n/2)
__device__ __forceinline__ int signed_mode(int i, int n) { return i < (n >> 1) ? i : i - n; }

__device__ __forceinline__ ModeQ mode_q(const DevPlan& p, int kx, int ky, int kz) {
    ModeQ m;
    const float qx = static_cast<float>(kx) * p.qs[0];
    const float qy = static_cast<float>(ky) * p.qs[1];
    const float qz = static_cast<float>(kz) * p.qs[2];
    m.q2 = qx * qx + qy * qy + qz * qz;
    m.iq[0] = (kx == -(p.n[0] >> 1)) ? 0.f : qx;
    m.iq[1] = (ky == -(p.n[1] >> 1)) ? 0.f : qy;
    m.iq[2] = (p.n[2] > 1 && kz == -(p.n[2] >> 1)) ? 0.f : qz;
    m.invq = m.q2 > 0.f ? 1.f / sqrtf(m.q2) : 0.f;
    return m;
}

// monomials with 1/|q| or i q_i factors, evaluated only by the kernel
// variants built for plans that have them
__device__ __forceinline__ float2 eval_general(const DevOp& op, const ModeQ& q) {
    const float q2 = q.q2, invq = q.invq, iqx = q.iq[0], iqy = q.iq[1], iqz = q.iq[2];
    float re = 0.f, im = 0.f;
    for (int i = 0; i < op.n; ++i) {
        const DevMono mo = op.m[i];
        float s = mo.coef;
        for (int e = 0; e < mo.q2; ++e) s *= q2;
        for (int e = 0; e < mo.invq; ++e) s *= invq;
        for (int e = 0; e < mo.ix; ++e) s *= iqx;
        for (int e = 0; e < mo.iy; ++e) s *= iqy;
        for (int e = 0; e < mo.iz; ++e) s *= iqz;
        switch (mo.ipow) {
            case 0: re += s; break;
            case 1: im += s; break;
            case 2: re -= s; break;
            default: im -= s; break;
        }
    }
    return make_float2(re, im);
}

// sum_j poly[j] (q^2)^j up to the operator's degree.  The coefficients are
// read at fixed offsets (no load waits for the degree) and the terms above
// the degree are skipped by a uniform branch; starting from r = 0 the first
// kept term gives r = poly[deg] exactly, as a loop from the degree would.
__device__ __forceinline__ float horner(const DevOp& op, float q2) {
    const int deg = op.deg;
    float r = 0.f;
#pragma unroll
    for (int j = PSS_MAXPOW; j >= 0; --j)
        if (j <= deg) r = fmaf(r, q2, op.poly[j]);
    return r;
}
// the same for P modes at once
template <int P>
__device__ __forceinline__ void horner_p(const DevOp& op, const float (&q2)[P], float (&out)[P]) {
    const int deg = op.deg;
#pragma unroll
    for (int m = 0; m < P; ++m) out[m] = 0.f;
#pragma unroll
    for (int j = PSS_MAXPOW; j >= 0; --j) {
        if (j <= deg) {
            const float c = op.poly[j];
#pragma unroll
            for (int m = 0; m < P; ++m) out[m] = fmaf(out[m], q2[m], c);
        }
    }
}

// sum_m coef (q^2)^a |q|^-b (i qx)^cx (i qy)^cy (i qz)^cz: Horner over the
// pure q^2 part, then the listed general monomials (GEN: the plan has some;
// without them the kernel is built without the out-of-line call, which would
// split the unrolled mode loops into separately scheduled pieces)
template <bool GEN>
__device__ __forceinline__ float2 eval_op(const DevOp& op, const ModeQ& q) {
    const float re = horner(op, q.q2);
    if constexpr (GEN) {
        if (op.n != 0) {
            const float2 g = eval_general(op, q);
            return make_float2(re + g.x, g.y);
        }
    }
    return make_float2(re, 0.f);
}

// 1 / (1 - dt L(q)), complex (operators with odd i q_i powers)
__device__ __forceinline__ float2 cinv_implicit(float dt, float2 L) {
    const float ar = 1.f - dt * L.x, ai = -dt * L.y;
    const float d = 1.f / (ar * ar + ai * ai);
    return make_float2(ar * d, -ai * d);
}

__device__ __forceinline__ bool mask_keep(const DevMask& mk, int kx, int ky, int kz) {
    if (mk.shape == 2) return true;
    if (mk.shape == 1) {
        bool k = true;
        if (mk.h[0]) k = k && (mk.den * abs(kx) < mk.num * mk.h[0]);
        if (mk.h[1]) k = k && (mk.den * abs(ky) < mk.num * mk.h[1]);
        if (mk.h[2]) k = k && (mk.den * abs(kz) < mk.num * mk.h[2]);
        return k;
    }
    const int64_t s = mk.w[0] * kx * kx + mk.w[1] * ky * ky + mk.w[2] * kz * kz;
    return s * mk.den2 < mk.rhs;
}

// Largest w^2 kept by mask mk along a line whose other indices are fixed at
// (kx, ky) (2D: kz is the line index; 3D lines run along z, 2D lines along
// y with kz absent): a mode of the line with index w is kept iff w*w <= lim.
// -1: the whole line is masked.  Decided once per line, exactly as
// mask_keep decides each mode.
template <int DIM>
__device__ __forceinline__ int line_lim(const DevMask& mk, int kx, int ky, int L) {
    const int hmax = (L >> 1) * (L >> 1);  // the largest w^2 on the line
    if (mk.shape == 2) return hmax;
    const int ia = DIM == 2 ? 1 : 2;  // axis of the line
    if (mk.shape == 1) {
        bool k = true;
        if (mk.h[0]) k = k && (mk.den * abs(kx) < mk.num * mk.h[0]);
        if (DIM == 3 && mk.h[1]) k = k && (mk.den * abs(ky) < mk.num * mk.h[1]);
        if (!k) return -1;
        if (!mk.h[ia]) return hmax;
        // den |w| < num h  <=>  |w| <= (num h - 1) / den
        const int wmax = (mk.num * mk.h[ia] - 1) / mk.den;
        return wmax * wmax;
    }
    // radial: (P0 + w_a w^2) den2 < rhs  <=>  w^2 <= (floor((rhs - 1)/den2) - P0) / w_a
    const int64_t p0 = mk.w[0] * kx * kx + (DIM == 3 ? mk.w[1] * ky * ky : 0);
    const int64_t room = (mk.rhs - 1) / mk.den2 - p0;
    if (room < 0) return -1;
    const int64_t wa = mk.w[ia];
    const int64_t lim = wa > 0 ? room / wa : hmax;
    return lim > hmax ? hmax : static_cast<int>(lim);
}

// Scaled unit white noise sigma(q) xi_hat(k) of field f at step `step` for a
// mode with full-spectrum linear index lin and negative-mode index lneg, and
// noise strength D(q) (Sec. "Adding noise").
__device__ __forceinline__ float2 noise_value(const DevPlan& p, int f, uint32_t step, uint32_t lin, uint32_t lneg,
                                              float D) {
    const uint32_t c = lin < lneg ? lin : lneg;
    const uint4 w = philox4x32_10(make_uint4(c, step, static_cast<uint32_t>(p.fid[f]), 0u), p.key0, p.key1);
    const float2 g = box_muller(w.x, w.y);
    const float sd = __builtin_amdgcn_sqrtf(fmaxf(D, 0.f));
    if (lin == lneg) return make_float2(p.amp_self * sd * g.x, 0.f);
    const float a = p.amp_pair * sd;
    return lin == c ? make_float2(a * g.x, a * g.y) : make_float2(a * g.x, -a * g.y);
}
template <bool GEN>
__device__ __forceinline__ float2 noise_mode(const DevPlan& p, int f, uint32_t step, uint32_t lin, uint32_t lneg,
                                             const ModeQ& q) {
    return noise_value(p, f, step, lin, lneg, eval_op<GEN>(p.noise_op[f], q).x);
}

// full-spectrum linear index of mode (kx, ky, kz), each in [0, n_i)
__device__ __forceinline__ uint32_t lin_index(const DevPlan& p, int kx, int ky, int kz) {
    return (static_cast<uint32_t>(kz) * p.n[1] + ky) * p.n[0] + kx;
}

// full-spectrum linear index and its negative for signed mode indices
__device__ __forceinline__ void mode_lin(const DevPlan& p, int kx, int ky, int kz, uint32_t& lin, uint32_t& lneg) {
    const int nx = p.n[0], ny = p.n[1], nz = p.n[2];
    const int ux = kx & (nx - 1), uy = ky & (ny - 1), uz = kz & (nz - 1);
    lin = lin_index(p, ux, uy, uz);
    lneg = lin_index(p, (nx - ux) & (nx - 1), (ny - uy) & (ny - 1), (nz - uz) & (nz - 1));
}

// f(integral_constant<int, I>) for I = 0 .. N-1, unrolled at compile time
template <int I, int N, class F>
__device__ __forceinline__ void static_for_from(F& f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for_from<I + 1, N>(f);
    }
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
    static_for_from<0, N>(f);
}

// Element f of a register array, f a runtime (block-uniform) field index.
// Written with bit masks rather than a chain of conditional copies: the
// compiler folds such a chain back into an indexed access, which moves the
// whole array to scratch memory.
template <int NF, int P>
__device__ __forceinline__ float2 pick(const float2 (&a)[NF][P], int f, int m) {
    if constexpr (NF == 1) return a[0][m];
    uint32_t rx = 0u, ry = 0u;
#pragma unroll
    for (int i = 0; i < NF; ++i) {
        const uint32_t mk = f == i ? 0xffffffffu : 0u;
        rx |= __float_as_uint(a[i][m].x) & mk;
        ry |= __float_as_uint(a[i][m].y) & mk;
    }
    return make_float2(__uint_as_float(rx), __uint_as_float(ry));
}

// a[f][m] += v, f a runtime field index: every element takes v or +0 (bit
// masks, for the reason given at pick)
template <int NF, int P>
__device__ __forceinline__ void add_to(float2 (&a)[NF][P], int f, int m, float2 v) {
    if constexpr (NF == 1) {
        if (f == 0) a[0][m] = cadd(a[0][m], v);
        return;
    }
#pragma unroll
    for (int i = 0; i < NF; ++i) {
        const uint32_t mk = f == i ? 0xffffffffu : 0u;
        a[i][m].x += __uint_as_float(__float_as_uint(v.x) & mk);
        a[i][m].y += __uint_as_float(__float_as_uint(v.y) & mk);
    }
}

// ------------------------------------------------------------ update kernel
// Lines along the last axis u (y in 2D, z in 3D).  A block holds TC packed
// columns x TO values of the other index o (y in 3D; none in 2D); the T
// threads of line (cc, lo) are consecutive, thread t keeps slot u = t + m*T
// of the line in v[m].  The state and the channel inputs are
// [o][ctile][u][TC]; the factor outputs V go to [ctile][u][TC] in 2D and to
// [u][ctile][o][TC] (the y-pass layout) in 3D.
//
// Which modes a line holds (signed indices):
//   c >= 1           : (c, u, -) in 2D, (c, o, u) in 3D
//   c = 0, 0<o<Ny/2  : (0, o, u)                          (3D)
//   c = 0, o>Ny/2    : (-Nx/2, Ny-o, u)                   (3D)
//   packed line (c = 0 in 2D; c = 0, o in {0, Ny/2} in 3D), slot form:
//     slot u in (0, L/2)  : kx = 0 at u
//     slot u in (L/2, L)  : kx = -Nx/2 at L - u
//     slots 0 and L/2     : (Re of kx = 0, Re of kx = -Nx/2), both real
// Transforms of a packed line see S(u) = phi(0,u) + i phi(Nx/2,u); the slot
// form is converted to and from it through one LDS line (block-uniform
// barriers; a block holds at most one packed line, its first).
// LDS: TC*TO line-transform regions | one exchange line of L | twiddles of L.

// packed line: S(u), S(L-u) -> slot value of u (the forward direction)
template <int L>
__device__ __forceinline__ float2 to_slot(int u, float2 a, float2 b) {
    if (u == 0 || u == (L >> 1)) return a;
    return u < (L >> 1) ? make_float2(0.5f * (a.x + b.x), 0.5f * (a.y - b.y))   // phi(0, u)
                        : make_float2(0.5f * (a.y + b.y), 0.5f * (a.x - b.x));  // phi(Nx/2, L-u)
}

// packed line: slot values of u and L-u -> S(u) = phi(0,u) + i phi(Nx/2,u)
template <int L>
__device__ __forceinline__ float2 from_slot(int u, float2 s1, float2 s2) {
    if (u == 0 || u == (L >> 1)) return s1;
    return u < (L >> 1) ? make_float2(s1.x - s2.y, s1.y + s2.x)   // phi0(u) + i phiN(u)
                        : make_float2(s2.x + s1.y, s1.x - s2.y);  // conj phi0(L-u) + i conj phiN(L-u)
}

// The modes of one line, decided once per thread: for slot u the signed
// index along the line is w(u), the fixed indices are those of the line
// (plain) or of the slot's half (packed: kx = 0 below L/2, -Nx/2 above).
struct LineModes {
    bool packed;
    int kx, ky;        // fixed indices of a plain line (3D: ky; 2D: ky unused)
    float qq;          // q_x^2 (+ q_y^2 in 3D) of a plain line
    float qqN;         // packed line: the same with kx = -Nx/2 (kx = 0 gives qq0)
    float qq0;
    float qs;          // q scale of the line axis
    uint32_t lstride;  // linear-index stride of the line axis
    uint32_t yx, yxn;  // linear-index parts of the fixed indices and of their negatives
    uint32_t yx0, yxN; // packed line: the same for kx = 0 and kx = -Nx/2 (negation keeps them)

};

// slot u (not a pair slot) of a line -> w, q^2, lin, lneg.  The line's
// description is taken by value so that it stays in registers.
template <int L>
__device__ __forceinline__ void slot_at(const LineModes lm, int u, float& q2, uint32_t& lin, uint32_t& lneg) {
    const bool upper = lm.packed && u > (L >> 1);
    const int w = lm.packed ? (upper ? L - u : u) : (u < (L >> 1) ? u : u - L);
    const float ql = static_cast<float>(w) * lm.qs;
    q2 = fmaf(ql, ql, lm.packed ? (upper ? lm.qqN : lm.qq0) : lm.qq);
    const uint32_t uw = static_cast<uint32_t>(w) & (L - 1), un = static_cast<uint32_t>(-w) & (L - 1);
    lin = uw * lm.lstride + (lm.packed ? (upper ? lm.yxN : lm.yx0) : lm.yx);
    lneg = un * lm.lstride + (lm.packed ? (upper ? lm.yxN : lm.yx0) : lm.yxn);
}

template <int L, int DIM>
__device__ __forceinline__ LineModes line_modes(const DevPlan& p, bool packed, int kx_l, int ky_l) {
    LineModes lm;
    const int nx = p.n[0], ny = p.n[1];
    lm.packed = packed;
    lm.kx = kx_l;
    lm.ky = ky_l;
    const float qx = static_cast<float>(kx_l) * p.qs[0];
    const float qy = DIM == 3 ? static_cast<float>(ky_l) * p.qs[1] : 0.f;
    const float qxN = static_cast<float>(nx >> 1) * p.qs[0];
    lm.qq = fmaf(qx, qx, qy * qy);
    lm.qq0 = qy * qy;
    lm.qqN = fmaf(qxN, qxN, qy * qy);
    lm.qs = p.qs[DIM == 2 ? 1 : 2];
    lm.lstride = DIM == 2 ? static_cast<uint32_t>(nx) : static_cast<uint32_t>(nx) * ny;
    const uint32_t ux = static_cast<uint32_t>(kx_l) & (nx - 1), uxn = static_cast<uint32_t>(-kx_l) & (nx - 1);
    const uint32_t uy = DIM == 3 ? (static_cast<uint32_t>(ky_l) & (ny - 1)) : 0u;
    const uint32_t uyn = DIM == 3 ? (static_cast<uint32_t>(-ky_l) & (ny - 1)) : 0u;
    lm.yx = uy * nx + ux;
    lm.yxn = uyn * nx + uxn;
    // packed lines: kx = 0 or Nx/2 are their own negatives (mod Nx); in 3D
    // the packed lines have ky = 0 or -Ny/2, also their own negatives
    lm.yx0 = uy * nx;
    lm.yxN = uy * nx + (nx >> 1);
    return lm;
}

// the two real self-conjugate modes (kx = 0 and kx = -Nx/2) of slot u in
// {0, L/2} of a packed line: signed index w of the line axis
template <int DIM>
__device__ __forceinline__ void pair_modes(int ky_l, int u, int L, int& ky, int& kz) {
    const int w = u == 0 ? 0 : -(L >> 1);
    if (DIM == 2) {
        ky = w;
        kz = 0;
    } else {
        ky = ky_l;
        kz = w;
    }
}

// op applied to a pair slot (re: kx = 0 mode, im: kx = -Nx/2 mode)
template <int DIM, bool GEN>
__device__ __forceinline__ float2 pair_op_d(const DevPlan& p, const DevOp& op, int ky_l, int u, int L, float2 a) {
    int ky, kz;
    pair_modes<DIM>(ky_l, u, L, ky, kz);
    return make_float2(eval_op<GEN>(op, mode_q(p, 0, ky, kz)).x * a.x,
                       eval_op<GEN>(op, mode_q(p, -(p.n[0] >> 1), ky, kz)).x * a.y);
}

// semi-implicit update of a pair slot
template <int DIM, bool GEN>
__device__ __forceinline__ float2 pair_update_d(const DevPlan& p, int f, uint32_t step, int ky_l, int u, int L,
                                                float2 old, float2 acc, bool noisy) {
    int ky, kz;
    pair_modes<DIM>(ky_l, u, L, ky, kz);
    const int kn = -(p.n[0] >> 1);
    const ModeQ q0 = mode_q(p, 0, ky, kz), qn = mode_q(p, kn, ky, kz);
    float2 r = cadd(old, cscale(acc, p.dt));
    if (noisy) {
        uint32_t lin, lneg;
        mode_lin(p, 0, ky, kz, lin, lneg);
        r.x += noise_mode<GEN>(p, f, step, lin, lneg, q0).x;
        mode_lin(p, kn, ky, kz, lin, lneg);
        r.y += noise_mode<GEN>(p, f, step, lin, lneg, qn).x;
    }
    return make_float2(r.x * cinv_implicit(p.dt, eval_op<GEN>(p.implicit_op[f], q0)).x,
                       r.y * cinv_implicit(p.dt, eval_op<GEN>(p.implicit_op[f], qn)).x);
}

// mode q of slot u of a line, for the general-monomial operators
template <int L, int DIM>
__device__ __forceinline__ ModeQ slot_q(const DevPlan& p, const LineModes lm, int u) {
    const bool upper = lm.packed && u > (L >> 1);
    const int w = lm.packed ? (upper ? L - u : u) : (u < (L >> 1) ? u : u - L);
    const int kx = lm.packed ? (upper ? -(p.n[0] >> 1) : 0) : lm.kx;
    return DIM == 2 ? mode_q(p, kx, w, 0) : mode_q(p, kx, lm.ky, w);
}

// slots 0 and L/2 of a packed line: op applied to their two real modes each
template <int DIM, bool GEN, int NF, int P>
__device__ __forceinline__ void pair_accumulate(float2 (&acc)[NF][P], int target, const float2 (&v)[P],
                                                const DevPlan& p, const DevOp& op, int ky_l, int L) {
    add_to(acc, target, 0, pair_op_d<DIM, GEN>(p, op, ky_l, 0, L, v[0]));
    add_to(acc, target, P / 2, pair_op_d<DIM, GEN>(p, op, ky_l, L >> 1, L, v[P / 2]));
}

// Fourier value of an intermediate field at the slots of one line, from the
// dynamic fields' values s there (Sec. "Writing models"):
//   psi = sum_k op_k(q) phi_{src_k} / (1 - L_psi(q)).
// On a packed line the pair slots come out in the same form as the state's:
// (value of the kx = 0 mode, value of the kx = -Nx/2 mode), both real, since
// every operator is real on those four self-conjugate modes.
template <int L, int P, int NF, int DIM>
__device__ __forceinline__ void interm_line(const DevPlan& p, const DevInterm& I, const float2 (&s)[NF][P],
                                            const LineModes lm, int t, bool pair_lane, int ky_l, float2 (&v)[P]) {
    constexpr int T = L / P;
    ModeQ q[P];
#pragma unroll
    for (int m = 0; m < P; ++m) {
        q[m] = slot_q<L, DIM>(p, lm, t + m * T);
        v[m] = make_float2(0.f, 0.f);
    }
    for (int k = 0; k < I.nsrc; ++k) {
        const int src = I.src[k];
#pragma unroll
        for (int m = 0; m < P; ++m) v[m] = cadd(v[m], cmul(eval_op<true>(I.op[k], q[m]), pick(s, src, m)));
    }
#pragma unroll
    for (int m = 0; m < P; ++m) v[m] = cmul(v[m], cinv_implicit(1.f, eval_op<true>(I.den, q[m])));
    if (pair_lane) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int mm = h ? P / 2 : 0;
            int ky, kz;
            pair_modes<DIM>(ky_l, h ? (L >> 1) : 0, L, ky, kz);
            const ModeQ q0 = mode_q(p, 0, ky, kz), qn = mode_q(p, -(p.n[0] >> 1), ky, kz);
            float re = 0.f, im = 0.f;
            for (int k = 0; k < I.nsrc; ++k) {
                const float2 a = pick(s, I.src[k], mm);
                re = fmaf(eval_op<true>(I.op[k], q0).x, a.x, re);
                im = fmaf(eval_op<true>(I.op[k], qn).x, a.y, im);
            }
            v[mm] = make_float2(re * cinv_implicit(1.f, eval_op<true>(I.den, q0)).x,
                                im * cinv_implicit(1.f, eval_op<true>(I.den, qn)).x);
        }
    }
}

// the values of factor or linear-term source `src` at the slots of a line:
// a dynamic field's own, or an intermediate's (only plans with the general
// operator code have intermediates)
template <int L, int P, int NF, int DIM, bool GEN>
__device__ __forceinline__ void source_line(const DevPlan& p, int src, const float2 (&s)[NF][P], const LineModes lm,
                                            int t, bool pair_lane, int ky_l, float2 (&v)[P]) {
    if constexpr (GEN) {
        if (src >= PSS_MAXF) {
            interm_line<L, P, NF, DIM>(p, p.interm[src - PSS_MAXF], s, lm, t, pair_lane, ky_l, v);
            return;
        }
    }
#pragma unroll
    for (int m = 0; m < P; ++m) v[m] = pick(s, src, m);
}

// One block of the update kernel: tile `blk` of lattice `mi`.  In the step
// modes of several lattices (TABLE) the lattice's buffers, counter and flag
// come from the member table and its plan from the plan array (both kernel
// arguments, so the plan reads stay scalar loads).  A launch of one lattice
// (and the transform modes) takes buffers, counter and flag from the
// arguments: its data loads then wait for no table load.
template <int L, int P, int NF, int MODE, int DIM, bool GEN, bool TABLE, int PADS = kFftPad>
__device__ __forceinline__ void update_block(int mi, int blk, const Member* __restrict__ members,
                                             const DevPlan* __restrict__ plans, const DevPlan* __restrict__ plan_a,
                                             const Bufs& bufs_a, const Geo& geo,
                                             const uint64_t* __restrict__ step_ctr_a, uint32_t* __restrict__ flag_a,
                                             int step_off, const float2* __restrict__ tw_g) {
    using FFT = LineFFT<L, P, PADS>;
    constexpr int T = FFT::T;
    extern __shared__ float2 smem[];
    constexpr bool TAB = (MODE == MODE_STEP || MODE == MODE_PROLOGUE) && TABLE;
    const Member* mem = members + mi;  // dereferenced in the step modes only
    // the lattice's plan, buffers and counter: from the tables or from the
    // arguments (selected at compile time, so the unused source is never
    // given an address)
    const DevPlan* pp;
    const Bufs* bp;
    const uint64_t* step_ctr;
    if constexpr (TAB) {
        pp = plans + mi;
        bp = &mem->bufs;
        step_ctr = mem->step_ctr;
    } else {
        pp = plan_a;
        bp = &bufs_a;
        step_ctr = step_ctr_a;
    }
    const DevPlan& p = *pp;
    const Bufs& bufs = *bp;
    const int tc = geo.tc, to = geo.to;
    const int ntile = geo.ntile;
    const int tid = threadIdx.x;
    const int nthr = tc * to * T;
    const int t = tid & (T - 1);
    const int li = tid / T;  // line of the block
    const int cc = li & (tc - 1);
    const int lo = li >> geo.tc_log2;
    const int ct = blk % ntile;  // tile index
    const int og = blk / ntile;  // group of `to` other-index lines
    const int o = og * to + lo;
    const int c = ct * tc + cc;  // packed column
    const int nx = p.n[0], ny = p.n[1];
    const size_t base = (static_cast<size_t>(o) * ntile + ct) * L * tc + cc;
    const size_t vbase = DIM == 2 ? base : (static_cast<size_t>(ct) * ny + o) * tc + cc;
    const size_t vstride = DIM == 2 ? static_cast<size_t>(tc) : static_cast<size_t>(ntile) * ny * tc;
    LdsLine ld;
    ld.wl = smem + li * FFT::kLds;
    ld.blk0 = ld.wl + FFT::kReg;
    ld.blk1 = ld.wl + 2 * FFT::kReg;
    ld.par = 0;
    float2* xbuf = smem + tc * to * FFT::kLds;  // packed-line exchange
    float2* twl = xbuf + L;
    const int dr = FFT::drev(t);  // gathered / scattered positions dr + m*T
    // twiddles: loaded now, stored to LDS after each mode's first loads
    float2 twr[P];
    load_twiddles<L, P>(twr, tw_g, tid, nthr);
    const float2* tw = twl;
    // block holds a packed line (block-uniform); this thread is on it
    const bool blk_packed = ct == 0 && (DIM == 2 || og * to == 0 || og * to == (ny >> 1));
    const bool packed = blk_packed && cc == 0 && lo == 0;
    const bool pair_lane = packed && t == 0;  // holds slots 0 and L/2: two real modes each
    // fixed mode indices of a plain line
    int kx_l = c, ky_l = 0;
    if (DIM == 3) {
        ky_l = signed_mode(o, ny);
        if (c == 0 && !packed) {
            if (o < (ny >> 1)) {
                kx_l = 0;
                ky_l = o;
            } else {
                kx_l = -(nx >> 1);
                ky_l = ny - o;
            }
        }
    }
    const int nf = p.nf;

    // packed line only: exchange v (natural order) with the partner slot -u
    // and map it (block-uniform)
    auto exchange = [&](float2 (&v)[P], bool forward) {
        if (!blk_packed) return;
        if (packed) {
#pragma unroll
            for (int m = 0; m < P; ++m) xbuf[t + m * T] = v[m];
        }
        __syncthreads();
        if (packed) {
#pragma unroll
            for (int m = 0; m < P; ++m) {
                const int u = t + m * T;
                const float2 b = xbuf[(L - u) & (L - 1)];
                v[m] = forward ? to_slot<L>(u, v[m], b) : from_slot<L>(u, v[m], b);
            }
        }
        __syncthreads();
    };

    if constexpr (MODE == MODE_FWD_STORE) {
        // forward transform of an array in the state layout, stored as the state
        float2 v[P];
#pragma unroll
        for (int m = 0; m < P; ++m) v[m] = gload(bufs.in + base + (dr + m * T) * tc);
        store_twiddles<L, P>(twl, twr, tid, nthr);
        __syncthreads();
        FFT::template dit<-1>(v, ld, t, tw);
        exchange(v, true);
#pragma unroll
        for (int m = 0; m < P; ++m) gstore(bufs.S[bufs.sel] + base + (t + m * T) * tc, v[m]);
        return;
    }
    if constexpr (MODE == MODE_INV_OUT) {
        float2 v[P];
#pragma unroll
        for (int m = 0; m < P; ++m) v[m] = gload(bufs.S[bufs.sel] + base + (t + m * T) * tc);
        store_twiddles<L, P>(twl, twr, tid, nthr);
        __syncthreads();
        exchange(v, false);
        FFT::template dif<1>(v, ld, t, tw);
#pragma unroll
        for (int m = 0; m < P; ++m) gstore(bufs.out + vbase + (dr + m * T) * vstride, v[m]);
        return;
    }

    // ---- MODE_STEP, MODE_PROLOGUE or MODE_INTERM_OUT
    const LineModes lmode = line_modes<L, DIM>(p, packed, kx_l, ky_l);
    float2 s[NF][P];  // state, then new state (slot form on a packed line)
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        if (f < nf) {
#pragma unroll
            for (int m = 0; m < P; ++m) s[f][m] = gload(bufs.S[f] + base + (t + m * T) * tc);
        } else {
#pragma unroll
            for (int m = 0; m < P; ++m) s[f][m] = make_float2(0.f, 0.f);
        }
    }

    if constexpr (MODE == MODE_INTERM_OUT) {
        // an intermediate field from the current state, inverse-transformed
        // along the line into `out` (natural order, as MODE_INV_OUT)
        store_twiddles<L, P>(twl, twr, tid, nthr);
        __syncthreads();
        float2 v[P];
        source_line<L, P, NF, DIM, GEN>(p, PSS_MAXF + bufs.sel, s, lmode, t, pair_lane, ky_l, v);
        exchange(v, false);
        FFT::template dif<1>(v, ld, t, tw);
#pragma unroll
        for (int m = 0; m < P; ++m) gstore(bufs.out + vbase + (dr + m * T) * vstride, v[m]);
        return;
    }
    if constexpr (MODE == MODE_PROLOGUE) {
        store_twiddles<L, P>(twl, twr, tid, nthr);
        __syncthreads();
    }
    if constexpr (MODE == MODE_STEP) {
        const uint32_t step = static_cast<uint32_t>(gload_u64(step_ctr)) + static_cast<uint32_t>(step_off);
        // the first channel's loads go out before the twiddles are stored
        float2 nxt[P];
        if (p.nch > 0) {
#pragma unroll
            for (int m = 0; m < P; ++m) nxt[m] = gload(bufs.N[0] + base + (t + m * T) * tc);
        }
        // per-slot modes of the line (slot form on a packed line)
        float q2[P];
        uint32_t lin[P], lneg[P];
#pragma unroll
        for (int m = 0; m < P; ++m) slot_at<L>(lmode, t + m * T, q2[m], lin[m], lneg[m]);
        // general operators: the mode vectors of the slots, once per line
        ModeQ qv[GEN ? P : 1];
        if constexpr (GEN) {
#pragma unroll
            for (int m = 0; m < P; ++m) qv[m] = slot_q<L, DIM>(p, lmode, t + m * T);
        }
        // the step's noise depends on the step and the modes only: formed
        // here, while the loads above are still in flight
        float2 eta[GEN ? 1 : NF][P];
        if constexpr (!GEN) {
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                if (f < nf && p.noisy[f] != 0) {
                    float Dn[P];
                    horner_p(p.noise_op[f], q2, Dn);
#pragma unroll
                    for (int m = 0; m < P; ++m) eta[f][m] = noise_value(p, f, step, lin[m], lneg[m], Dn[m]);
                } else {
#pragma unroll
                    for (int m = 0; m < P; ++m) eta[f][m] = make_float2(0.f, 0.f);
                }
            }
        }
        store_twiddles<L, P>(twl, twr, tid, nthr);  // waits for the twiddle loads
        __syncthreads();  // twiddles in LDS
        float2 acc[NF][P];  // explicit contributions
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int m = 0; m < P; ++m) acc[f][m] = make_float2(0.f, 0.f);
        // explicit real-space channels: forward transform, then M(q) per mode
        for (int ch = 0; ch < p.nch; ++ch) {
            const DevChannel& C = p.ch[ch];
            float2 v[P];
#pragma unroll
            for (int m = 0; m < P; ++m) v[m] = nxt[m];
            if (ch + 1 < p.nch) {
#pragma unroll
                for (int m = 0; m < P; ++m) nxt[m] = gload(bufs.N[ch + 1] + base + (t + m * T) * tc);
            }
            FFT::template dit<-1>(v, ld, t, tw);
            exchange(v, true);
            // each output: its operator times the transform, into its field
            // (one field: one output, so the loop is left out)
            const int nout = NF == 1 ? 1 : C.nout;
            for (int o = 0; o < nout; ++o) {
                const DevOp& op = C.op[o];
                const int tg = C.target[o];
                if constexpr (GEN) {
#pragma unroll
                    for (int m = 0; m < P; ++m)
                        if (!(pair_lane && (m == 0 || m == P / 2)))
                            add_to(acc, tg, m, cmul(eval_op<GEN>(op, qv[m]), v[m]));
                } else {
                    float M[P];
                    horner_p(op, q2, M);
#pragma unroll
                    for (int m = 0; m < P; ++m)
                        if (!(pair_lane && (m == 0 || m == P / 2))) add_to(acc, tg, m, cscale(v[m], M[m]));
                }
                // slots 0 and L/2 of a packed line: two real modes (operators are real on them)
                if (pair_lane) pair_accumulate<DIM, GEN>(acc, tg, v, p, op, ky_l, L);
            }
        }
        // Fourier-space terms with a single linear factor
        for (int d = 0; d < p.nd; ++d) {
            const DevDirect& Dd = p.direct[d];
            float2 src[P];  // from the step-n state (an intermediate: its step-n value)
            source_line<L, P, NF, DIM, GEN>(p, Dd.src, s, lmode, t, pair_lane, ky_l, src);
            if constexpr (GEN) {
#pragma unroll
                for (int m = 0; m < P; ++m)
                    if (!(pair_lane && (m == 0 || m == P / 2)))
                        add_to(acc, Dd.target, m, cmul(eval_op<GEN>(Dd.op, qv[m]), src[m]));
            } else {
                float M[P];
                horner_p(Dd.op, q2, M);
#pragma unroll
                for (int m = 0; m < P; ++m)
                    if (!(pair_lane && (m == 0 || m == P / 2))) add_to(acc, Dd.target, m, cscale(src[m], M[m]));
            }
            if (pair_lane) pair_accumulate<DIM, GEN>(acc, Dd.target, src, p, Dd.op, ky_l, L);
        }
        // semi-implicit update (eq:timeupdate) with in-register noise
        // fields unrolled by template: a loop that the compiler leaves rolled
        // (the general-operator bodies are large) indexes s and acc at run
        // time, which moves both arrays to scratch memory
        uint32_t bad = 0;
        static_for<NF>([&](auto FF) {
            constexpr int f = decltype(FF)::value;
            if (f >= nf) return;
            const bool noisy = p.noisy[f] != 0;
            const float2 old0 = s[f][0], oldh = s[f][P / 2];
            float Ar[P];
            if constexpr (!GEN) horner_p(p.implicit_op[f], q2, Ar);
#pragma unroll
            for (int m = 0; m < P; ++m) {
                float2 r = cadd(s[f][m], cscale(acc[f][m], p.dt));
                if constexpr (GEN) {
                    const ModeQ& q = qv[m];
                    if (noisy) r = cadd(r, noise_mode<GEN>(p, f, step, lin[m], lneg[m], q));
                    s[f][m] = cmul(r, cinv_implicit(p.dt, eval_op<GEN>(p.implicit_op[f], q)));
                } else {
                    if (noisy) r = cadd(r, eta[f][m]);
                    s[f][m] = cscale(r, __builtin_amdgcn_rcpf(fmaf(-p.dt, Ar[m], 1.f)));
                }
            }
            if (pair_lane) {
                // slots 0 and L/2 hold two real modes each
                s[f][0] = pair_update_d<DIM, GEN>(p, f, step, ky_l, 0, L, old0, acc[f][0], noisy);
                s[f][P / 2] = pair_update_d<DIM, GEN>(p, f, step, ky_l, L >> 1, L, oldh, acc[f][P / 2], noisy);
            }
            bool fin = true;
#pragma unroll
            for (int m = 0; m < P; ++m) {
                gstore_sel<!TABLE>(bufs.S[f] + base + (t + m * T) * tc, s[f][m]);
                fin = fin && __builtin_isfinite(s[f][m].x) && __builtin_isfinite(s[f][m].y);
            }
            if (!fin) bad |= 1u << f;  // a NaN or infinity in the new state
        });
        if (bad) {
            if constexpr (TAB) {
                atomicOr(mem->flag, bad);
            } else {
                atomicOr(flag_a, bad);
            }
        }
    }

    // de-aliased inverse transforms of every factor field (eq:cubicexampledealiased)
    for (int g = 0; g < p.ng; ++g) {
        const DevMask& mk = p.mask[g];
        if (ct * tc >= mk.ncol) continue;  // whole tile masked: never read (block-uniform)
        // the factor's Fourier values (a dynamic field's new state, or an
        // intermediate computed from it)
        float2 a[P];
        source_line<L, P, NF, DIM, GEN>(p, p.gfield[g], s, lmode, t, pair_lane, ky_l, a);
        // the largest kept w^2 of this line (packed: of each half)
        const int lim = line_lim<DIM>(mk, lmode.packed ? 0 : kx_l, ky_l, L);
        const int limN = line_lim<DIM>(mk, -(nx >> 1), ky_l, L);
        float2 v[P];
#pragma unroll
        for (int m = 0; m < P; ++m) {
            const int u = t + m * T;
            const bool upper = packed && u > (L >> 1);
            const int w = packed ? (upper ? L - u : u) : (u < (L >> 1) ? u : u - L);
            v[m] = w * w <= (upper ? limN : lim) ? a[m] : make_float2(0.f, 0.f);
        }
        if (pair_lane) {
            // slots 0 and L/2: kx = 0 (re) and kx = -Nx/2 (im) at w = 0, -L/2
            const int wh = (L >> 1) * (L >> 1);
            const float2 a0 = a[0], ah = a[P / 2];
            v[0] = make_float2(0 <= lim ? a0.x : 0.f, 0 <= limN ? a0.y : 0.f);
            v[P / 2] = make_float2(wh <= lim ? ah.x : 0.f, wh <= limN ? ah.y : 0.f);
        }
        exchange(v, false);
        FFT::template dif<1>(v, ld, t, tw);
#pragma unroll
        for (int m = 0; m < P; ++m) gstore_sel<!TABLE>(bufs.V[g] + vbase + (t + m * T) * vstride, v[m]);
    }
}

template <int L, int P, int NF, int MODE, int DIM, bool GEN, bool TABLE>
__global__ void __launch_bounds__(256) update_kernel(const Member* __restrict__ members,
                                                      const DevPlan* __restrict__ plans,
                                                      const DevPlan* __restrict__ plan_a, Bufs bufs_a, Geo geo,
                                                      const uint64_t* __restrict__ step_ctr_a,
                                                      uint32_t* __restrict__ flag_a, int step_off,
                                                      const float2* __restrict__ tw_g) {
    // lattice blockIdx.y, XCD-ordered over the whole grid
    const int nb = gridDim.x;
    const int lin_b = xcd_block(blockIdx.y * nb + blockIdx.x, nb * gridDim.y);
    const int mi = lin_b / nb;
    update_block<L, P, NF, MODE, DIM, GEN, TABLE>(mi, lin_b - mi * nb, members, plans, plan_a, bufs_a, geo,
                                                  step_ctr_a, flag_a, step_off, tw_g);
}

// ------------------------------------------------------ adjoint column kernel
// One reverse step of 2D Model B along y lines (AdjArgs).  Same block shape,
// slot form and LDS layout as the 2D update kernel: TC column lines per
// block, the T threads of a line consecutive, thread t holds slots
// u = t + m*T.  Inner products over all modes become sums over the stored
// slots with weight 2 (a mode and its conjugate), and weight 1 for each real
// component of the pair slots.
template <int L, int P, int MODE>
__global__ void __launch_bounds__(256) adjcol_kernel(AdjArgs aa, Geo geo, const float2* __restrict__ tw_g) {
    using FFT = LineFFT<L, P>;
    constexpr int T = FFT::T;
    extern __shared__ float2 smem[];
    const DevPlan& p = *aa.plan;
    const int tc = geo.tc;
    const int tid = threadIdx.x;
    const int nthr = tc * T;
    const int t = tid & (T - 1);
    const int cc = tid / T;
    const int ct = xcd_block(blockIdx.x, gridDim.x);
    const int c = ct * tc + cc;
    const int nx = p.n[0];
    const int kn = -(nx >> 1);
    const size_t base = static_cast<size_t>(ct) * L * tc + cc;
    LdsLine ld;
    ld.wl = smem + cc * FFT::kLds;
    ld.blk0 = ld.wl + FFT::kReg;
    ld.blk1 = ld.wl + 2 * FFT::kReg;
    ld.par = 0;
    float2* xbuf = smem + tc * FFT::kLds;
    float2* twl = xbuf + L;
    const int dr = FFT::drev(t);
    float2 twr[P];
    load_twiddles<L, P>(twr, tw_g, tid, nthr);
    const float2* tw = twl;
    const bool blk_packed = ct == 0;
    const bool packed = blk_packed && cc == 0;
    const DevMask& mk = p.mask[0];

    auto exchange = [&](float2 (&v)[P], bool forward) {  // as in the update kernel
        if (!blk_packed) return;
        if (packed) {
#pragma unroll
            for (int m = 0; m < P; ++m) xbuf[t + m * T] = v[m];
        }
        __syncthreads();
        if (packed) {
#pragma unroll
            for (int m = 0; m < P; ++m) {
                const int u = t + m * T;
                const float2 b = xbuf[(L - u) & (L - 1)];
                v[m] = forward ? to_slot<L>(u, v[m], b) : from_slot<L>(u, v[m], b);
            }
        }
        __syncthreads();
    };
    // modes of slot u: (kx, ky) of a plain slot, or pair = the two real modes
    auto slot = [&](int u, int& kx, int& ky, bool& pair) {
        pair = false;
        if (!packed) {
            kx = c;
            ky = signed_mode(u, L);
        } else if (u == 0 || u == (L >> 1)) {
            pair = true;
            kx = 0;
            ky = u == 0 ? 0 : -(L >> 1);
        } else if (u < (L >> 1)) {
            kx = 0;
            ky = u;
        } else {
            kx = kn;
            ky = L - u;
        }
    };

    // g_{n+1}
    float2 g[P];
    if (aa.first) {
#pragma unroll
        for (int m = 0; m < P; ++m) g[m] = aa.G[base + (t + m * T) * tc];
        store_twiddles<L, P>(twl, twr, tid, nthr);
        __syncthreads();
    } else {
        float2 v[P];
#pragma unroll
        for (int m = 0; m < P; ++m) v[m] = aa.X[base + (t + m * T) * tc];
        store_twiddles<L, P>(twl, twr, tid, nthr);
        __syncthreads();
        FFT::template dit<-1>(v, ld, t, tw);
        exchange(v, true);
#pragma unroll
        for (int m = 0; m < P; ++m) {
            int kx, ky;
            bool pair;
            slot(t + m * T, kx, ky, pair);
            float2 y = cscale(v[m], p.inv_n * aa.b);
            if (!pair) {
                if (!mask_keep(mk, kx, ky, 0)) y = make_float2(0.f, 0.f);
            } else {
                if (!mask_keep(mk, 0, ky, 0)) y.x = 0.f;
                if (!mask_keep(mk, kn, ky, 0)) y.y = 0.f;
            }
            g[m] = cadd(aa.Rin[base + (t + m * T) * tc], y);
        }
    }
    if constexpr (MODE == MODE_ADJFIN) {
#pragma unroll
        for (int m = 0; m < P; ++m) aa.Rout[base + (t + m * T) * tc] = g[m];
        return;
    }

    // r_n = g_{n+1} / A, the coefficient sums, -dt q^2 r_n and m phi_n
    const float dt = p.dt;
    const bool noisy = p.noisy[0] != 0;
    double part[3] = {0.0, 0.0, 0.0};  // d/da, d/dk, <r, eta>
    float2 wr[P], um[P];
#pragma unroll
    for (int m = 0; m < P; ++m) {
        const int u = t + m * T;
        const size_t e = base + u * tc;
        int kx, ky;
        bool pair;
        slot(u, kx, ky, pair);
        const float2 f1 = aa.phi1[e], f0 = aa.phi0[e];
        float2 r;
        if (!pair) {
            const ModeQ q = mode_q(p, kx, ky, 0);
            r = cscale(g[m], 1.f / (1.f + dt * q.q2 * (aa.a + aa.k * q.q2)));
            const double re1 = static_cast<double>(r.x) * f1.x + static_cast<double>(r.y) * f1.y;
            part[0] -= 2.0 * dt * q.q2 * re1;
            part[1] -= 2.0 * dt * static_cast<double>(q.q2) * q.q2 * re1;
            if (noisy) {
                uint32_t lin, lneg;
                mode_lin(p, kx, ky, 0, lin, lneg);
                const float2 eta = noise_mode<false>(p, 0, aa.step, lin, lneg, q);
                part[2] += 2.0 * (static_cast<double>(r.x) * eta.x + static_cast<double>(r.y) * eta.y);
            }
            wr[m] = cscale(r, -dt * q.q2);
            um[m] = mask_keep(mk, kx, ky, 0) ? f0 : make_float2(0.f, 0.f);
        } else {
            // two real modes: re part kx = 0, im part kx = -Nx/2
            const ModeQ q0 = mode_q(p, 0, ky, 0), qn = mode_q(p, kn, ky, 0);
            r = make_float2(g[m].x / (1.f + dt * q0.q2 * (aa.a + aa.k * q0.q2)),
                            g[m].y / (1.f + dt * qn.q2 * (aa.a + aa.k * qn.q2)));
            const double e0 = static_cast<double>(r.x) * f1.x, en = static_cast<double>(r.y) * f1.y;
            part[0] -= dt * (q0.q2 * e0 + qn.q2 * en);
            part[1] -= dt * (static_cast<double>(q0.q2) * q0.q2 * e0 + static_cast<double>(qn.q2) * qn.q2 * en);
            if (noisy) {
                uint32_t lin, lneg;
                mode_lin(p, 0, ky, 0, lin, lneg);
                const float eta0 = noise_mode<false>(p, 0, aa.step, lin, lneg, q0).x;
                mode_lin(p, kn, ky, 0, lin, lneg);
                const float etan = noise_mode<false>(p, 0, aa.step, lin, lneg, qn).x;
                part[2] += static_cast<double>(r.x) * eta0 + static_cast<double>(r.y) * etan;
            }
            wr[m] = make_float2(-dt * q0.q2 * r.x, -dt * qn.q2 * r.y);
            um[m] = make_float2(mask_keep(mk, 0, ky, 0) ? f0.x : 0.f, mask_keep(mk, kn, ky, 0) ? f0.y : 0.f);
        }
        aa.Rout[e] = r;
    }
    exchange(wr, false);
    FFT::template dif<1>(wr, ld, t, tw);
#pragma unroll
    for (int m = 0; m < P; ++m) aa.W[base + (t + m * T) * tc] = wr[m];
    exchange(um, false);
    FFT::template dif<1>(um, ld, t, tw);
#pragma unroll
    for (int m = 0; m < P; ++m) aa.U[base + (t + m * T) * tc] = um[m];
    if (aa.D > 0.f) part[2] /= 2.0 * aa.D;
    block_sum_to_slot(part, aa.acc + static_cast<size_t>(blockIdx.x) * 3);
}

#if defined(PSS_COMMON)
// terminal seed of the adjoint: g(k) = coef[shell(k)] phi(k) on the 2D packed
// state layout (slot form on column 0), shell(k) = rint(|k|)
__global__ void adjseed_kernel(const float2* __restrict__ phi, float2* __restrict__ g, const float* __restrict__ coef,
                               int nshell, int nx, int ny, int tc) {
    const int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const int64_t total = static_cast<int64_t>(nx / 2) * ny;
    if (e >= total) return;
    const int cc = static_cast<int>(e % tc);
    const int y = static_cast<int>((e / tc) % ny);
    const int col = static_cast<int>(e / (static_cast<int64_t>(tc) * ny)) * tc + cc;
    auto cf = [&](int kx, int ky) {
        const int j = static_cast<int>(rintf(sqrtf(static_cast<float>(kx * kx + ky * ky))));
        return (j >= 1 && j < nshell) ? coef[j] : 0.f;
    };
    const float2 v = phi[e];
    float2 o;
    if (col > 0) {
        const float s = cf(col, y < ny / 2 ? y : y - ny);
        o = make_float2(s * v.x, s * v.y);
    } else if (y == 0 || y == ny / 2) {
        const int w = y == 0 ? 0 : -(ny / 2);
        o = make_float2(cf(0, w) * v.x, cf(-(nx / 2), w) * v.y);
    } else if (y < ny / 2) {
        const float s = cf(0, y);
        o = make_float2(s * v.x, s * v.y);
    } else {
        const float s = cf(-(nx / 2), ny - y);
        o = make_float2(s * v.x, s * v.y);
    }
    g[e] = o;
}
#endif  // PSS_COMMON

// ----------------------------------------------------------------- y pass
// 3D only: lines along y for fixed (c, z); block = TC columns x TZ values of
// z, the T threads of a line consecutive.  Input [z][ctile][y][TC].  The
// inverse pass writes the same layout, the forward pass writes the state
// layout [y][ctile][z][TC].
//
// Column 0 arrives from the x pass as X(0) + i X(Nx/2), both real; after the
// forward y transform it is Y(ky) = Y0(ky) + i YN(ky) with Y0, YN Hermitian
// in ky.  The forward pass re-packs it so that every z line of column 0
// except ky = 0, Ny/2 holds single modes:
//   slot ky in (0, Ny/2)   : Y0(ky)          (modes kx = 0)
//   slot Ny-ky             : YN(ky)          (modes kx = Nx/2)
//   slots 0 and Ny/2       : Y unchanged     (packed, Hermitian along z)
// and the inverse pass undoes it before transforming.
template <int L, int P, int MODE>
__global__ void __launch_bounds__(256) ypass_kernel(YArgs ya, Geo geo, const float2* __restrict__ tw_g) {
    using FFT = LineFFT<L, P>;
    constexpr int T = FFT::T;
    extern __shared__ float2 smem[];
    const int tc = geo.tc, tz = geo.tz;
    const int ntile = geo.ntile;
    const int nz = geo.nz;
    const int tid = threadIdx.x;
    const int nthr = tc * tz * T;
    const int t = tid & (T - 1);
    const int li = tid / T;
    const int cc = li & (tc - 1);
    const int lz = li >> geo.tc_log2;
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int ct = blk % ntile;
    const int z = (blk / ntile) * tz + lz;
    const int c = ct * tc + cc;
    LdsLine ld;
    ld.wl = smem + li * FFT::kLds;
    ld.blk0 = ld.wl + FFT::kReg;
    ld.blk1 = ld.wl + 2 * FFT::kReg;
    ld.par = 0;
    float2* xb = smem + tc * tz * FFT::kLds + lz * L;  // column-0 exchange, one line per z
    const int dr = FFT::drev(t);
    float2 twr[P];
    load_twiddles<L, P>(twr, tw_g, tid, nthr);
    const float2* tw = store_twiddles<L, P>(smem + tc * tz * FFT::kLds + tz * L, twr, tid, nthr);
    __syncthreads();
    const size_t ibase = (static_cast<size_t>(z) * ntile + ct) * L * tc + cc;
    const size_t obase = MODE == MODE_YFWD ? (static_cast<size_t>(ct) * nz + z) * tc + cc : ibase;
    const size_t ostride = MODE == MODE_YFWD ? static_cast<size_t>(ntile) * nz * tc : static_cast<size_t>(tc);

    for (int a = 0; a < ya.n; ++a) {
        if (ct * tc >= ya.ncol[a]) continue;  // tile holds no kept column (block-uniform)
        const float2* __restrict__ src = ya.src[a];
        float2* __restrict__ dst = ya.dst[a];
        float2 v[P];
        if constexpr (MODE == MODE_YINV) {
            // gathered at the digit-reversed positions, natural order out
#pragma unroll
            for (int m = 0; m < P; ++m) {
                const int y = dr + m * T;
                const float2 s1 = src[ibase + y * tc];
                if (c == 0 && y != 0 && y != (L >> 1)) {
                    const float2 s2 = src[ibase + (L - y) * tc];
                    v[m] = y < (L >> 1) ? make_float2(s1.x - s2.y, s1.y + s2.x)   // Y0 + i YN
                                        : make_float2(s2.x + s1.y, s1.x - s2.y);  // conj(Y0) + i conj(YN)
                } else {
                    v[m] = s1;
                }
            }
            // in place (src == dst) is safe: a line is read whole before any of
            // it is written, within one wave or across the transform's barrier
            FFT::template dit<1>(v, ld, t, tw);
#pragma unroll
            for (int m = 0; m < P; ++m) dst[obase + (t + m * T) * ostride] = v[m];
        } else {
#pragma unroll
            for (int m = 0; m < P; ++m) v[m] = src[ibase + (t + m * T) * tc];
            FFT::template dif<-1>(v, ld, t, tw);
            if (ct == 0) {
                // column 0: the partner of ky is L - ky, exchanged by natural position
                if (c == 0) {
#pragma unroll
                    for (int m = 0; m < P; ++m) xb[dr + m * T] = v[m];
                }
                __syncthreads();
                if (c == 0) {
#pragma unroll
                    for (int m = 0; m < P; ++m) {
                        const int y = dr + m * T;
                        if (y == 0 || y == (L >> 1)) continue;
                        const float2 a0 = v[m], b0 = xb[L - y];
                        v[m] = y < (L >> 1) ? make_float2(0.5f * (a0.x + b0.x), 0.5f * (a0.y - b0.y))   // Y0(y)
                                            : make_float2(0.5f * (a0.y + b0.y), 0.5f * (a0.x - b0.x));  // YN(L-y)
                    }
                }
                __syncthreads();
            }
#pragma unroll
            for (int m = 0; m < P; ++m) dst[obase + (dr + m * T) * ostride] = v[m];
        }
    }
}

// ----------------------------------------------------------------- x kernel
// Rows of length L = Nx; block = RB consecutive rows, pair pr = rows
// (2 pr, 2 pr + 1) packed as one complex line held by T consecutive threads.
// Packed-column arrays are read and written in whole tile blocks of RB*TC
// contiguous elements.
// One block of the x kernel: row block `blk` of lattice `mi` (as in the update kernel)
template <int L, int P, int NG, int MODE, bool TABLE, int PADS = kFftPad>
__device__ __forceinline__ void xrow_block(int mi, int blk, const Member* __restrict__ members,
                                           const DevPlan* __restrict__ plans, const DevPlan* __restrict__ plan_a,
                                           const Bufs& bufs_a, const Geo& geo, const float2* __restrict__ tw_g,
                                           int64_t advance, uint64_t* __restrict__ step_ctr_a) {
    using FFT = LineFFT<L, P, PADS>;
    constexpr int T = FFT::T;
    constexpr int NC = L / 2;  // packed columns
    extern __shared__ float2 smem[];
    constexpr bool TAB = MODE == MODE_STEP && TABLE;  // as in the update kernel
    const Member* mem = members + mi;
    const DevPlan* pp;
    const Bufs* bp;
    if constexpr (TAB) {
        pp = plans + mi;
        bp = &mem->bufs;
    } else {
        pp = plan_a;
        bp = &bufs_a;
    }
    const DevPlan& p = *pp;
    const Bufs& bufs = *bp;
    const int tc = geo.tc, rb = geo.rb;
    const int ntile = NC / tc;
    const int tid = threadIdx.x;
    const int nthr = (rb >> 1) * T;
    const int pr = tid / T;  // pair within the block
    const int t = tid & (T - 1);
    const int r0 = blk * rb;  // first row; row index = z*Ny + y
    const int ny = p.n[1];
    const int zr = r0 / ny;          // z of the block (0 in 2D)
    const int y0 = r0 - zr * ny;     // first y of the block
    const int lt = geo.tc_log2;
    LdsLine ld;
    ld.wl = smem + pr * FFT::kLds;
    ld.blk0 = ld.wl + FFT::kReg;
    ld.blk1 = ld.wl + 2 * FFT::kReg;
    ld.par = 0;
    const int dr = FFT::drev(t);
    // twiddles: loaded now, stored to LDS after each mode's first loads
    float2 twr[P];
    load_twiddles<L, P>(twr, tw_g, tid, nthr);
    float2* const twl = smem + (rb >> 1) * FFT::kLds;
    const float2* tw = twl;

    // Gather the packed complex input Z[k] = X_row0[k] + i X_row1[k] of pair
    // pr at k = dr + m T straight from the packed-column array (columns
    // [0, ncol) are stored; the others are zero); all loads are issued together.
    const size_t row0 = (static_cast<size_t>(zr) * ntile * ny + y0 + 2 * pr) * tc;
    const size_t tstride = static_cast<size_t>(ny) * tc;  // one column tile
    auto build_z = [&](float2 (&v)[P], const float2* __restrict__ src, int ncol) {
        // all loads first, without control flow between them; a dropped
        // column reads column 0 and then counts as zero
        float2 a[P], b[P];
        if (tc == 1) {
            // one-column tiles: the pair's two rows are neighbours, and the
            // row pair starts at an even row, so one aligned 16-byte load
            // takes both (half the address work of two 8-byte loads)
#pragma unroll
            for (int m = 0; m < P; ++m) {
                const int k = dr + m * T;
                const int kk = (k == NC) ? 0 : (k < NC ? k : L - k);
                const int kc = kk < ncol ? kk : 0;
                gload_pair(src + row0 + kc * tstride, a[m], b[m]);
            }
        } else {
#pragma unroll
            for (int m = 0; m < P; ++m) {
                const int k = dr + m * T;
                const int kk = (k == NC) ? 0 : (k < NC ? k : L - k);
                const int kc = kk < ncol ? kk : 0;
                const size_t off = row0 + (kc >> lt) * tstride + (kc & (tc - 1));
                a[m] = gload(src + off);
                b[m] = gload(src + off + tc);
            }
        }
#pragma unroll
        for (int m = 0; m < P; ++m) {
            const int k = dr + m * T;
            const int kk = (k == NC) ? 0 : (k < NC ? k : L - k);
            const float2 zero = make_float2(0.f, 0.f);
            const float2 am = kk < ncol ? a[m] : zero, bm = kk < ncol ? b[m] : zero;
            float2 z;
            if (k == 0) {
                z = make_float2(am.x, bm.x);
            } else if (k == NC) {
                z = make_float2(am.y, bm.y);
            } else {
                z = k < NC ? make_float2(am.x - bm.y, am.y + bm.x) : make_float2(am.x + bm.y, bm.x - am.y);
            }
            v[m] = z;
        }
    };
    // Stage the forward transform W (held at k = dr + m T) of every pair in
    // LDS at its natural positions, then unpack the two real rows of each
    // pair and store whole packed-column tiles.  A line wider than a wave
    // stages in its next block buffer; a narrower one in its own region
    // (its wave is done with it).  The caller separates consecutive calls by
    // a block barrier when the staging region is the in-wave one.
    auto store_rows = [&](const float2 (&w)[P], float2* __restrict__ dst) {
        float2* stage = FFT::kCross ? ld.next_blk() : ld.wl;
        if constexpr (!FFT::kCross) wave_lds_sync();  // after the transform's last in-wave reads
#pragma unroll
        for (int m = 0; m < P; ++m) stage[dr + m * T] = w[m];
        __syncthreads();
        const int lp = geo.rb_log2 + lt;  // log2(rb * tc)
        const int total = ntile << lp;
        const size_t sbase = (static_cast<size_t>(zr) * ntile) * ny + y0;
#pragma unroll 4
        for (int i = tid; i < total; i += nthr) {
            const int tl = i >> lp, rem = i & ((1 << lp) - 1);
            const int r = rem >> lt, cc = rem & (tc - 1);
            const int c = (tl << lt) + cc;
            const float2* W = smem + (r >> 1) * FFT::kLds + (FFT::kCross ? (stage - ld.wl) : 0);
            float2 o;
            if (c == 0) {
                const float2 a = W[0], b = W[NC];
                o = (r & 1) ? make_float2(a.y, b.y) : make_float2(a.x, b.x);
            } else {
                const float2 a = W[c], b = W[L - c];
                o = (r & 1) ? make_float2(0.5f * (a.y + b.y), 0.5f * (b.x - a.x))
                            : make_float2(0.5f * (a.x + b.x), 0.5f * (a.y - b.y));
            }
            gstore_sel<!TABLE>(dst + ((sbase + static_cast<size_t>(tl) * ny + r) << lt) + cc, o);
        }
    };

    if constexpr (MODE == MODE_R2C_IN) {
        // real rows -> packed columns (forward transform, unnormalised)
        const float* __restrict__ src = bufs.real_in;
        float2 v[P];
#pragma unroll
        for (int m = 0; m < P; ++m) {
            const int x = t + m * T;
            v[m] = make_float2(src[static_cast<size_t>(r0 + 2 * pr) * L + x],
                               src[static_cast<size_t>(r0 + 2 * pr + 1) * L + x]);
        }
        store_twiddles<L, P>(twl, twr, tid, nthr);
        __syncthreads();
        FFT::template dif<-1>(v, ld, t, tw);
        store_rows(v, bufs.out);
        return;
    }
    if constexpr (MODE == MODE_C2R_OUT) {
        float2 v[P];
        build_z(v, bufs.in, NC);
        store_twiddles<L, P>(twl, twr, tid, nthr);
        __syncthreads();
        FFT::template dit<1>(v, ld, t, tw);
        float* __restrict__ dst = bufs.real_out;
#pragma unroll
        for (int m = 0; m < P; ++m) {
            const int x = t + m * T;
            dst[static_cast<size_t>(r0 + 2 * pr) * L + x] = v[m].x * p.inv_n;
            dst[static_cast<size_t>(r0 + 2 * pr + 1) * L + x] = v[m].y * p.inv_n;
        }
        return;
    }

    if constexpr (MODE == MODE_ADJROW) {
        // reverse step, real space: u = F^-1[m phi_n] (rows of V[0], kept
        // columns only), w = N F^-1[-dt q^2 r] (rows of V[1], unnormalised),
        // 3 u^2 w -> forward x transform into N[0] (the column kernel applies
        // the factor b); and the FP64 sum of u^3 w, which is
        // <r, -dt q^2 F[u^3]> = dL/db of the step, by Parseval
        float2 u[P], w[P];
        build_z(u, bufs.V[0], p.mask[0].ncol);
        build_z(w, bufs.V[1], p.mask[1].ncol);
        store_twiddles<L, P>(twl, twr, tid, nthr);
        __syncthreads();
        FFT::template dit<1>(u, ld, t, tw);
        FFT::template dit<1>(w, ld, t, tw);
        double part[1] = {0.0};
#pragma unroll
        for (int m = 0; m < P; ++m) {
            const float ux = u[m].x * p.inv_n, uy = u[m].y * p.inv_n;
            part[0] += static_cast<double>(ux) * ux * ux * w[m].x + static_cast<double>(uy) * uy * uy * w[m].y;
            u[m] = make_float2(3.f * ux * ux * w[m].x, 3.f * uy * uy * w[m].y);
        }
        FFT::template dif<-1>(u, ld, t, tw);
        store_rows(u, bufs.N[0]);
        block_sum_to_slot(part, bufs.acc + blockIdx.x);
        return;
    }

    // MODE_STEP: the last step of a replayed chunk moves the member's step
    // counter on (no later kernel of the chunk reads it)
    if (advance != 0 && r0 == 0 && tid == 0) {
        if constexpr (TAB) {
            *mem->step_ctr += static_cast<uint64_t>(advance);
        } else {
            *step_ctr_a += static_cast<uint64_t>(advance);
        }
    }
    // real-space values of every factor field (the variant with room for
    // more than four holds zeros in the slots beyond the plan's)
    float2 z[NG][P];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        if (NG > 4 && g >= p.ng) {
#pragma unroll
            for (int m = 0; m < P; ++m) z[g][m] = make_float2(0.f, 0.f);
            continue;
        }
        float2 v[P];
        build_z(v, bufs.V[g], p.mask[g].ncol);
        if (g == 0) {
            store_twiddles<L, P>(twl, twr, tid, nthr);
            __syncthreads();
        }
        FFT::template dit<1>(v, ld, t, tw);
#pragma unroll
        for (int m = 0; m < P; ++m) z[g][m] = cscale(v[m], p.inv_n);
    }
    // products per channel, forward transform, store
    for (int ch = 0; ch < p.nch; ++ch) {
        const DevChannel& C = p.ch[ch];
        float2 w[P];
#pragma unroll
        for (int m = 0; m < P; ++m) w[m] = make_float2(0.f, 0.f);
        for (int k = 0; k < C.nprod; ++k) {
            const DevProd& pd = C.prod[k];
            // the factor powers read as one 64-bit word (a scalar load)
            static_assert(sizeof(pd.pow) == 8, "eight factor slots");
            uint64_t pw;
            __builtin_memcpy(&pw, pd.pow, sizeof(pw));
#pragma unroll
            for (int m = 0; m < P; ++m) {
                float a = pd.coef, b = pd.coef;
#pragma unroll
                for (int g = 0; g < NG; ++g) {
                    const int pg = static_cast<int>((pw >> (8 * g)) & 0xffull);
                    for (int e = 0; e < pg; ++e) {
                        a *= z[g][m].x;
                        b *= z[g][m].y;
                    }
                }
                w[m].x += a;
                w[m].y += b;
            }
        }
        if (!FFT::kCross && ch > 0) __syncthreads();  // the previous channel's rows are stored
        FFT::template dif<-1>(w, ld, t, tw);
        store_rows(w, bufs.N[ch]);
    }
}

template <int L, int P, int NG, int MODE, bool TABLE>
__global__ void __launch_bounds__(256) xrow_kernel(const Member* __restrict__ members,
                                                    const DevPlan* __restrict__ plans,
                                                    const DevPlan* __restrict__ plan_a, Bufs bufs_a, Geo geo,
                                                    const float2* __restrict__ tw_g, int64_t advance,
                                                    uint64_t* __restrict__ step_ctr_a) {
    const int nb = gridDim.x;
    const int lin_b = xcd_block(blockIdx.y * nb + blockIdx.x, nb * gridDim.y);
    const int mi = lin_b / nb;
    xrow_block<L, P, NG, MODE, TABLE>(mi, lin_b - mi * nb, members, plans, plan_a, bufs_a, geo, tw_g, advance,
                                      step_ctr_a);
}

#if defined(PSS_COMMON)
// ---------------------------------------------------------------- utilities
__global__ void advance_kernel(uint64_t* step_ctr, int64_t k) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *step_ctr += static_cast<uint64_t>(k);
}

__global__ void advance_many_kernel(uint64_t* const* __restrict__ ctrs, int n, int64_t k) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) *ctrs[i] += static_cast<uint64_t>(k);
}

// a boundary frame on a real-space array: site frame[i].x takes the value
// whose bits are frame[i].y
__global__ void apply_frame_kernel(float* __restrict__ real, const int2* __restrict__ frame, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) {
        const int2 e = frame[i];
        real[e.x] = __int_as_float(e.y);
    }
}

// read and clear the non-finite flag that follows each member's step counter
__global__ void take_flags_kernel(uint64_t* const* __restrict__ ctrs, int n, uint32_t* __restrict__ out) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = atomicExch(reinterpret_cast<uint32_t*>(ctrs[i] + 1), 0u);
}

__global__ void init_uniform_kernel(float* __restrict__ out, int64_t n, uint32_t field, uint32_t key0,
                                    uint32_t key1, double lo, double hi) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint4 w = philox4x32_10(make_uint4(static_cast<uint32_t>(i), 0u, field, 1u), key0, key1);
    const double u = (static_cast<double>(w.x >> 9) + 0.5) * 1.1920928955078125e-07;
    out[i] = static_cast<float>(__dadd_rn(lo, __dmul_rn(hi - lo, u)));
}

__global__ void philox_kernel(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                              int64_t count, uint32_t* __restrict__ out) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const uint4 w = philox4x32_10(make_uint4(c0 + static_cast<uint32_t>(i), c1, c2, c3), k0, k1);
    reinterpret_cast<uint4*>(out)[i] = w;
}


// Shell sums for the structure factor.  Thread i handles packed element i of
// the 2D tiled layout [ctile][y][TC]; interior columns stand for the mode and
// its conjugate partner (weight 2); column 0 is unpacked into kx = 0 and
// kx = Nx/2 (weight 1 each) with the partner element at -y.  With dim = 1 the
// array is a full spectrum, element (kz Ny + ky) Nx + kx for mode (kx, ky, kz)
// (weight 1): 1D lines and mixed-radix 2D and 3D lattices.  shell_terms calls
// emit(j, t) for every term t = w * scale * |phi_hat|^2 of shell j.
//
// The sums are exact, so they do not depend on the order in which the
// threads and blocks add: a first pass takes the largest binary exponent E_j
// of the terms of each shell (a max, order-free), a second adds every term
// as the integer round(t * 2^(61 - e_j)) (e_j = E_j - 1023, so each is below
// 2^62) into a 128-bit accumulator (64-bit atomics with carry; integer sums
// are associative), and a last pass turns the integer back into a double.
// Each term is rounded once, to 2^-62 of the shell's largest term.
template <typename F>
__device__ __forceinline__ void shell_terms(const float2* __restrict__ S, int64_t e, int nx, int ny, int nz, int tc,
                                            int dim, int nshell, double scale, F&& emit) {
    auto mag = [](float2 v) { return static_cast<double>(v.x) * v.x + static_cast<double>(v.y) * v.y; };
    auto add = [&](int kx, int ky, int kz, double v, int w) {
        const double kk = static_cast<double>(kx) * kx + static_cast<double>(ky) * ky + static_cast<double>(kz) * kz;
        const int j = static_cast<int>(rint(sqrt(kk)));
        if (j >= 1 && j < nshell) emit(j, scale * v * w, static_cast<unsigned int>(w));
    };
    if (dim == 1) {
        // a full complex spectrum (1D lines, mixed-radix 2D and 3D
        // lattices): each mode once
        const int kx = static_cast<int>(e % nx), ky = static_cast<int>((e / nx) % ny),
                  kz = static_cast<int>(e / (static_cast<int64_t>(nx) * ny));
        add(kx < nx / 2 ? kx : kx - nx, ny == 1 ? 0 : (ky < ny / 2 ? ky : ky - ny),
            nz == 1 ? 0 : (kz < nz / 2 ? kz : kz - nz), mag(S[e]), 1);
        return;
    }
    const int ncols = nx / 2;
    const int ntile = ncols / tc;
    const int cc = static_cast<int>(e % tc);
    const int64_t r = e / tc;
    int c, y, z;
    if (dim == 2) {
        y = static_cast<int>(r % ny);
        c = static_cast<int>(r / ny) * tc + cc;
        z = 0;
    } else {
        z = static_cast<int>(r % nz);
        const int64_t r2 = r / nz;
        c = static_cast<int>(r2 % ntile) * tc + cc;
        y = static_cast<int>(r2 / ntile);
    }
    const int ky = y < ny / 2 ? y : y - ny;
    const int kz = nz == 1 ? 0 : (z < nz / 2 ? z : z - nz);
    const float2 a = S[e];
    if (c > 0) {
        add(c, ky, kz, mag(a), 2);
        return;
    }
    // column 0: slot form along the update axis on packed lines
    const bool packed = dim == 2 || y == 0 || y == ny / 2;
    if (!packed) {
        if (y < ny / 2)
            add(0, y, kz, mag(a), 2);
        else
            add(-(nx / 2), ny - y, kz, mag(a), 2);
        return;
    }
    const int L = dim == 2 ? ny : nz;
    const int u = dim == 2 ? y : z;
    const int ky0 = dim == 2 ? 0 : ky;
    auto at = [&](int w) { return dim == 2 ? make_int2(w, 0) : make_int2(ky0, w); };  // (ky, kz) of index w
    if (u == 0 || u == L / 2) {
        const int w = u == 0 ? 0 : -(L / 2);
        const int2 yz = at(w);
        add(0, yz.x, yz.y, static_cast<double>(a.x) * a.x, 1);
        add(-(nx / 2), yz.x, yz.y, static_cast<double>(a.y) * a.y, 1);
    } else if (u < L / 2) {
        const int2 yz = at(u);
        add(0, yz.x, yz.y, mag(a), 2);
    } else {
        const int2 yz = at(L - u);
        add(-(nx / 2), yz.x, yz.y, mag(a), 2);
    }
}

// order key of a term: twice its biased exponent, +1 for a NaN (so that a
// NaN wins over an infinity, as it would in a plain sum)
__device__ __forceinline__ unsigned int shell_key(double t) {
    const unsigned long long b = static_cast<unsigned long long>(__double_as_longlong(t));
    const unsigned int E = static_cast<unsigned int>((b >> 52) & 0x7ffull);
    const bool nan = E == 0x7ffu && (b & 0xfffffffffffffull) != 0ull;
    return 2u * E + (nan ? 1u : 0u);
}

__device__ __forceinline__ int64_t shell_total(int nx, int ny, int nz, int dim) {
    return dim == 1 ? static_cast<int64_t>(nx) * ny * nz : static_cast<int64_t>(nx / 2) * ny * nz;
}

// pass 1: key[j] = max over the terms of shell j
__global__ void shell_keys_kernel(const float2* __restrict__ S, int nx, int ny, int nz, int tc, int dim, double scale,
                                  int nshell, unsigned int* __restrict__ gkey) {
    extern __shared__ unsigned int lkey[];
    for (int i = threadIdx.x; i < nshell; i += blockDim.x) lkey[i] = 0u;
    __syncthreads();
    const int64_t total = shell_total(nx, ny, nz, dim);
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x)
        shell_terms(S, e, nx, ny, nz, tc, dim, nshell, scale,
                    [&](int j, double t, unsigned int) { atomicMax(&lkey[j], shell_key(t)); });
    __syncthreads();
    for (int i = threadIdx.x; i < nshell; i += blockDim.x)
        if (lkey[i]) atomicMax(&gkey[i], lkey[i]);
}

// 128-bit add of (hi, lo) into (*h, *l) with 64-bit atomics
__device__ __forceinline__ void add128(unsigned long long* h, unsigned long long* l, unsigned long long hi,
                                       unsigned long long lo) {
    const unsigned long long old = atomicAdd(l, lo);
    hi += old + lo < old ? 1ull : 0ull;
    if (hi) atomicAdd(h, hi);
}

// pass 2: the exact fixed-point sums and the shell populations
__global__ void shell_sums_kernel(const float2* __restrict__ S, int nx, int ny, int nz, int tc, int dim, double scale,
                                  int nshell, const unsigned int* __restrict__ gkey, unsigned long long* __restrict__ ghi,
                                  unsigned long long* __restrict__ glo, unsigned long long* __restrict__ gcnt) {
    extern __shared__ unsigned long long lacc[];
    unsigned long long* lhi = lacc;
    unsigned long long* llo = lacc + nshell;
    unsigned int* lcnt = reinterpret_cast<unsigned int*>(lacc + 2 * nshell);
    unsigned int* lkey = lcnt + nshell;
    for (int i = threadIdx.x; i < nshell; i += blockDim.x) {
        lhi[i] = 0ull;
        llo[i] = 0ull;
        lcnt[i] = 0u;
        lkey[i] = gkey[i];
    }
    __syncthreads();
    const int64_t total = shell_total(nx, ny, nz, dim);
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x)
        shell_terms(S, e, nx, ny, nz, tc, dim, nshell, scale, [&](int j, double t, unsigned int w) {
            atomicAdd(&lcnt[j], w);
            const int E = static_cast<int>(lkey[j] >> 1);
            if (E == 0x7ff || t == 0.0) return;  // a non-finite shell is settled by its key
            add128(&lhi[j], &llo[j], 0ull, __double2ull_rn(ldexp(t, 1084 - E)));
        });
    __syncthreads();
    for (int i = threadIdx.x; i < nshell; i += blockDim.x) {
        if (lcnt[i]) {
            add128(&ghi[i], &glo[i], lhi[i], llo[i]);
            atomicAdd(&gcnt[i], static_cast<unsigned long long>(lcnt[i]));
        }
    }
}

// pass 3: shell means S_j = sum_j / count_j, written over hi[j] as doubles
__global__ void shell_means_kernel(int nshell, const unsigned int* __restrict__ gkey,
                                   unsigned long long* __restrict__ ghi, const unsigned long long* __restrict__ glo,
                                   const unsigned long long* __restrict__ gcnt) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nshell) return;
    const unsigned int key = gkey[j];
    const int E = static_cast<int>(key >> 1);
    double v;
    if (E == 0x7ff) {
        v = (key & 1u) ? __longlong_as_double(0x7ff8000000000000ll) : __longlong_as_double(0x7ff0000000000000ll);
    } else {
        const double m = static_cast<double>(ghi[j]) * 18446744073709551616.0 + static_cast<double>(glo[j]);
        v = ldexp(m, E - 1084);
    }
    const unsigned long long n = gcnt[j];
    ghi[j] = static_cast<unsigned long long>(__double_as_longlong(n ? v / static_cast<double>(n) : 0.0));
}

// ------------------------------------------- 1D lines of mixed-radix length
// Lines whose length N = 2^a 3^b 5^c (a >= 1) is not a power of two.  One
// block per lattice keeps the spectra in LDS and transforms them with
// self-sorting (Stockham) passes of radix 4, 2, 3 and 5 (Van Loan, Sec. 1.7):
// a pass of radix r over the current length n = m r and s interleaved
// transforms maps x to
//   y[q + s (r p + j)] = w_n^(j p) sum_l x[q + s (p + l m)] w_r^(j l),
// p < m, q < s, j < r, w_n = exp(-+2 pi i / n), and the next pass takes n = m,
// s = s r, until the result stands in natural order.  The step is the one of
// the power-of-two 1D kernel, mode by mode over the whole line.

// (cos, sin)(2 pi k / r) for r in {2, 3, 4, 5}
__device__ __forceinline__ float2 small_root(int r, int k) {
    // the fifth roots: cos and sin of 72 and 144 degrees
    constexpr float c1 = 0.309016994374947424f, s1 = 0.951056516295153572f;
    constexpr float c2 = -0.809016994374947424f, s2 = 0.587785252292473129f;
    constexpr float h3 = 0.866025403784438647f;  // sin(120 degrees)
    switch (r) {
        case 2: return k == 0 ? make_float2(1.f, 0.f) : make_float2(-1.f, 0.f);
        case 3: return k == 0 ? make_float2(1.f, 0.f) : (k == 1 ? make_float2(-0.5f, h3) : make_float2(-0.5f, -h3));
        case 4:
            return k == 0 ? make_float2(1.f, 0.f)
                          : (k == 1 ? make_float2(0.f, 1.f) : (k == 2 ? make_float2(-1.f, 0.f) : make_float2(0.f, -1.f)));
        default:
            switch (k) {
                case 0: return make_float2(1.f, 0.f);
                case 1: return make_float2(c1, s1);
                case 2: return make_float2(c2, s2);
                case 3: return make_float2(c2, -s2);
                default: return make_float2(c1, -s1);
            }
    }
}

// floor(x / d) for 0 <= x < 2^21 and d >= 1, without an integer division:
// (x + 1/2)/d lies at least 1/(2d) from an integer, and rounding 1/d and the
// product moves it by less than 2^-22 (x + 1/2)/d, below 1/(2d) for such x,
// so truncating the FP32 product gives the exact quotient
struct FastDiv {
    int d;
    float rd;
    __device__ __forceinline__ explicit FastDiv(int dv) : d(dv), rd(1.0f / static_cast<float>(dv)) {}
    __device__ __forceinline__ int quo(int x) const {
        return static_cast<int>((static_cast<float>(x) + 0.5f) * rd);
    }
};

// One self-sorting pass of radix R over nl lines of N values (line l at
// x + l N), sign sg = -1 (forward) or +1 (inverse): the radix-R transforms of
// the current length n = m R, then the twiddles w_n^(j p).  n s = N at every
// pass, so j p s < N indexes the table directly.  Lines hold at most 2^21
// values in all (they sit in LDS).
template <int R>
__device__ __forceinline__ void mr_pass(const float2* __restrict__ x, float2* __restrict__ y,
                                        const float2* __restrict__ tw, int N, int m, int s, int nl, float sg) {
    const int per = m * s;
    const FastDiv fper(per), fs(s);
    for (int idx = threadIdx.x; idx < nl * per; idx += blockDim.x) {
        const int line = fper.quo(idx), rem = idx - line * per;
        const int p = fs.quo(rem), q = rem - p * s;
        const float2* xl = x + static_cast<size_t>(line) * N;
        float2* yl = y + static_cast<size_t>(line) * N;
        float2 a[R];
#pragma unroll
        for (int l = 0; l < R; ++l) a[l] = xl[q + s * (p + l * m)];
#pragma unroll
        for (int j = 0; j < R; ++j) {
            float2 b = a[0];
#pragma unroll
            for (int l = 1; l < R; ++l) {
                float2 w = small_root(R, (j * l) % R);
                w.y *= sg;
                b = cadd(b, cmul(a[l], w));
            }
            if (j > 0) {
                float2 w = tw[j * p * s];  // exp(-2 pi i j p s / N) = w_n^(j p)
                if (sg > 0.f) w.y = -w.y;
                b = cmul(b, w);
            }
            yl[q + s * (R * p + j)] = b;
        }
    }
}

// Transform of nl lines of N values in x (LDS; line l at x + l N) with sign
// -1 (forward) or +1 (inverse, unnormalised); y is LDS scratch of the same
// size.  Returns the buffer holding the result.  Every thread of the block
// calls it; it ends with a barrier.
__device__ float2* mr_transform(float2* x, float2* y, const float2* __restrict__ tw, const MrPlan& mr, int sign,
                                int nl = 1) {
    const int N = mr.n;
    const float sg = static_cast<float>(sign);
    int n = N, s = 1;
    for (int st = 0; st < mr.nst; ++st) {
        const int r = mr.radix[st];
        const int m = n / r;
        switch (r) {
            case 4: mr_pass<4>(x, y, tw, N, m, s, nl, sg); break;
            case 2: mr_pass<2>(x, y, tw, N, m, s, nl, sg); break;
            case 3: mr_pass<3>(x, y, tw, N, m, s, nl, sg); break;
            default: mr_pass<5>(x, y, tw, N, m, s, nl, sg); break;
        }
        __syncthreads();
        float2* t = x;
        x = y;
        y = t;
        n = m;
        s *= r;
    }
    return x;
}

template <int NF, bool GEN, int MODE>
__global__ void __launch_bounds__(256)
    line1d_mr_kernel(const DevPlan* __restrict__ plan, Bufs bufs, uint64_t* __restrict__ step_ctr,
                     uint32_t* __restrict__ flag, int nsteps, int advance, const float2* __restrict__ tw_g, MrPlan mr) {
    extern __shared__ float2 smem[];
    const DevPlan& p = *plan;
    const int N = mr.n;
    const int t = threadIdx.x, T = blockDim.x;
    float2* const tw = smem;         // exp(-2 pi i k / N)
    float2* const A = smem + N;      // transform buffers
    float2* const B = smem + 2 * N;
    float2* const S = smem + 3 * N;  // states [NF][N]
    float2* const acc = S + NF * N;  // explicit contributions [NF][N]
    float* const u = reinterpret_cast<float*>(acc + NF * N);  // de-aliased factors [ng][N]
    for (int i = t; i < N; i += T) tw[i] = tw_g[i];
    auto kq = [&](int k) { return mode_q(p, k < (N >> 1) ? k : k - N, 0, 0); };

    if constexpr (MODE == MODE_FWD_STORE) {
        for (int i = t; i < N; i += T) A[i] = make_float2(bufs.real_in[i], 0.f);
        __syncthreads();
        const float2* r = mr_transform(A, B, tw, mr, -1);
        for (int k = t; k < N; k += T) gstore(bufs.S[bufs.sel] + k, r[k]);
        return;
    }
    if constexpr (MODE == MODE_INV_OUT) {
        for (int k = t; k < N; k += T) A[k] = gload(bufs.S[bufs.sel] + k);
        __syncthreads();
        const float2* r = mr_transform(A, B, tw, mr, 1);
        for (int i = t; i < N; i += T) bufs.real_out[i] = r[i].x * p.inv_n;
        return;
    }

    const int nf = p.nf;
    for (int f = 0; f < nf; ++f)
        for (int k = t; k < N; k += T) S[f * N + k] = gload(bufs.S[f] + k);
    __syncthreads();
    // Fourier value of source src (a dynamic field, or an intermediate
    // psi = sum_j op_j phi_j / (1 - L_psi)) at mode k of the current state
    auto source = [&](int src, int k, const ModeQ& q) -> float2 {
        if constexpr (GEN) {
            if (src >= PSS_MAXF) {
                const DevInterm& I = p.interm[src - PSS_MAXF];
                float2 v = make_float2(0.f, 0.f);
                for (int j = 0; j < I.nsrc; ++j) v = cadd(v, cmul(eval_op<true>(I.op[j], q), S[I.src[j] * N + k]));
                return cmul(v, cinv_implicit(1.f, eval_op<true>(I.den, q)));
            }
        }
        return S[src * N + k];
    };

    if constexpr (MODE == MODE_INTERM_OUT) {
        for (int k = t; k < N; k += T) A[k] = source(PSS_MAXF + bufs.sel, k, kq(k));
        __syncthreads();
        const float2* r = mr_transform(A, B, tw, mr, 1);
        for (int i = t; i < N; i += T) bufs.real_out[i] = r[i].x * p.inv_n;
        return;
    }

    // MODE_STEP: acc = sum_ch M_ch(q) F[products] from the current state
    auto channels = [&]() {
        for (int i = t; i < nf * N; i += T) acc[i] = make_float2(0.f, 0.f);
        if (p.nch == 0) {
            __syncthreads();
            return;
        }
        for (int g = 0; g < p.ng; ++g) {
            const DevMask& mk = p.mask[g];
            for (int k = t; k < N; k += T)
                A[k] = mask_keep(mk, k < (N >> 1) ? k : k - N, 0, 0) ? source(p.gfield[g], k, kq(k))
                                                                     : make_float2(0.f, 0.f);
            __syncthreads();
            const float2* r = mr_transform(A, B, tw, mr, 1);
            for (int i = t; i < N; i += T) u[g * N + i] = r[i].x * p.inv_n;
            __syncthreads();
        }
        for (int ch = 0; ch < p.nch; ++ch) {
            const DevChannel& C = p.ch[ch];
            for (int i = t; i < N; i += T) {
                float w = 0.f;
                for (int k = 0; k < C.nprod; ++k) {
                    const DevProd& pd = C.prod[k];
                    float a = pd.coef;
                    for (int g = 0; g < p.ng; ++g)
                        for (int e = 0; e < pd.pow[g]; ++e) a *= u[g * N + i];
                    w += a;
                }
                A[i] = make_float2(w, 0.f);
            }
            __syncthreads();
            const float2* r = mr_transform(A, B, tw, mr, -1);
            for (int k = t; k < N; k += T) {
                const ModeQ q = kq(k);
                for (int o = 0; o < C.nout; ++o) {
                    float2& d = acc[C.target[o] * N + k];
                    d = cadd(d, cmul(eval_op<GEN>(C.op[o], q), r[k]));
                }
            }
            __syncthreads();
        }
    };

    const uint32_t step0 = static_cast<uint32_t>(gload_u64(step_ctr));
    uint32_t bad = 0;
    channels();
    for (int sn = 0; sn < nsteps; ++sn) {
        const uint32_t step = step0 + static_cast<uint32_t>(sn);
        // linear explicit terms from the step-n state, then the semi-implicit
        // update with the noise of this step (each mode by one thread)
        for (int k = t; k < N; k += T) {
            const ModeQ q = kq(k);
            for (int d = 0; d < p.nd; ++d) {
                const DevDirect& Dd = p.direct[d];
                float2& a = acc[Dd.target * N + k];
                a = cadd(a, cmul(eval_op<GEN>(Dd.op, q), source(Dd.src, k, q)));
            }
        }
        __syncthreads();  // the intermediates of the direct terms read every field's step-n state
        for (int k = t; k < N; k += T) {
            const ModeQ q = kq(k);
            const uint32_t lin = static_cast<uint32_t>(k), lneg = static_cast<uint32_t>((N - k) % N);
            for (int f = 0; f < nf; ++f) {
                float2 r = cadd(S[f * N + k], cscale(acc[f * N + k], p.dt));
                if (p.noisy[f] != 0) r = cadd(r, noise_mode<GEN>(p, f, step, lin, lneg, q));
                r = cmul(r, cinv_implicit(p.dt, eval_op<GEN>(p.implicit_op[f], q)));
                S[f * N + k] = r;
                if (!(__builtin_isfinite(r.x) && __builtin_isfinite(r.y))) bad |= 1u << f;
            }
        }
        __syncthreads();
        // boundary frames: the new state's real space takes the frame values
        // on the frame sites, then is transformed back
        for (int f = 0; f < nf; ++f) {
            if (p.nframe[f] == 0) continue;
            for (int k = t; k < N; k += T) A[k] = S[f * N + k];
            __syncthreads();
            float2* r = mr_transform(A, B, tw, mr, 1);
            float2* o = r == A ? B : A;
            for (int i = t; i < N; i += T) o[i] = make_float2(r[i].x * p.inv_n, 0.f);
            __syncthreads();
            const int2* __restrict__ fr = p.frame[f];
            for (int i = t; i < p.nframe[f]; i += T) o[fr[i].x] = make_float2(__int_as_float(fr[i].y), 0.f);
            __syncthreads();
            const float2* z = mr_transform(o, r, tw, mr, -1);
            for (int k = t; k < N; k += T) S[f * N + k] = z[k];
            __syncthreads();
        }
        if (sn + 1 < nsteps) channels();
    }
    for (int f = 0; f < nf; ++f)
        for (int k = t; k < N; k += T) gstore(bufs.S[f] + k, S[f * N + k]);
    if (bad) atomicOr(flag, bad);
    __syncthreads();  // every thread has read the counter
    if (advance && t == 0) *step_ctr += static_cast<uint64_t>(nsteps);
}

hipError_t launch_line1d_mr(int mode, int N, int nf, int ng, const LaunchArgs& a) {
    MrPlan mr{};
    if (!mr_plan(N, &mr)) return hipErrorInvalidValue;
    const int NF = nf <= 1 ? 1 : (nf == 2 ? 2 : 4);
    const size_t lds = line1d_mr_lds_bytes(mr.n, NF, ng);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    const dim3 grid(1), block(256);
    uint64_t* ctr = const_cast<uint64_t*>(a.step_ctr);
    const bool gen = a.general || mode == MODE_INTERM_OUT;
#define PSS_MR(NFV, G, M)                                                                                   \
    hipLaunchKernelGGL((line1d_mr_kernel<NFV, G, M>), grid, block, lds, a.stream, a.plan, a.bufs, ctr, a.flag, \
                       a.nsteps, a.advance != 0 ? 1 : 0, a.tw_x, mr)
#define PSS_MRF(M)                       \
    do {                                 \
        if (NF == 1) {                   \
            if (gen)                     \
                PSS_MR(1, true, M);      \
            else                         \
                PSS_MR(1, false, M);     \
        } else if (NF == 2) {            \
            if (gen)                     \
                PSS_MR(2, true, M);      \
            else                         \
                PSS_MR(2, false, M);     \
        } else {                         \
            if (gen)                     \
                PSS_MR(4, true, M);      \
            else                         \
                PSS_MR(4, false, M);     \
        }                                \
    } while (0)
    switch (mode) {
        case MODE_STEP: PSS_MRF(MODE_STEP); break;
        case MODE_INTERM_OUT: PSS_MRF(MODE_INTERM_OUT); break;
        case MODE_FWD_STORE: PSS_MR(1, false, MODE_FWD_STORE); break;
        case MODE_INV_OUT: PSS_MR(1, false, MODE_INV_OUT); break;
        default: return hipErrorInvalidValue;
    }
#undef PSS_MRF
#undef PSS_MR
    return hipGetLastError();
}

hipError_t line1d_mr_setup() {
    const int lds = 160 * 1024;
#define PSS_MRA(NFV, G, M)                                                                                     \
    if (hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&line1d_mr_kernel<NFV, G, M>),        \
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds))                   \
        return e;
#define PSS_MRB(M) PSS_MRA(1, false, M) PSS_MRA(1, true, M) PSS_MRA(2, false, M) PSS_MRA(2, true, M) \
    PSS_MRA(4, false, M) PSS_MRA(4, true, M)
    PSS_MRB(MODE_STEP)
    PSS_MRB(MODE_INTERM_OUT)
    PSS_MRA(1, false, MODE_FWD_STORE)
    PSS_MRA(1, false, MODE_INV_OUT)
#undef PSS_MRB
#undef PSS_MRA
    return hipSuccess;
}

// ------------------------------- 2D and 3D lattices of mixed-radix sizes
// Every size an even 2^a 3^b 5^c, at least one not a power of two.  The state
// of a field is its full complex spectrum, mode (kx, ky, kz) at
// (kz Ny + ky) Nx + kx (natural order on every axis); real space is the real
// part of the inverse transform, as everywhere.  A step is launched as on the
// power-of-two path: the column kernel (one block per line along the last
// axis: forward transforms of the channels, the update, the de-aliased
// factors' inverse transforms), in 3D a y pass, the row kernel (one block per
// x row: inverse x transforms of the factors, the real-space products, their
// forward x transforms), in 3D a y pass back; each line in LDS and
// transformed with the self-sorting passes above.

template <int NF, bool GEN, int MODE>
__global__ void __launch_bounds__(256)
    mr2_col_kernel(const DevPlan* __restrict__ plan, Bufs bufs, const uint64_t* __restrict__ step_ctr,
                   uint32_t* __restrict__ flag, int step_off, const float2* __restrict__ tw_g, MrPlan my, int tc) {
    extern __shared__ float2 smem[];
    const DevPlan& p = *plan;
    // tc neighbouring lines along the last axis: y in 2D (block = kx0 ..
    // kx0 + tc - 1), z in 3D (the same kx range at one ky); "ky" below is the
    // index along a line.  LDS holds line c of an array at c L.
    const int Nx = p.n[0], L = my.n, N1 = p.n[1];
    const bool d3 = p.n[2] > 1;
    const int nxb = Nx / tc;
    // XCD-ordered blocks: each XCD's L2 takes a contiguous range of columns,
    // so the cache lines that neighbouring column blocks share are fetched
    // into one L2, not into all eight
    const int blk = xcd_block(blockIdx.x, gridDim.x);
    const int kx0 = (blk % nxb) * tc;
    const int ko = d3 ? blk / nxb : 0;  // ky of 3D lines
    const int kos = ko < (N1 >> 1) ? ko : ko - N1;
    const size_t base = d3 ? static_cast<size_t>(ko) * Nx + kx0 : static_cast<size_t>(kx0);
    const size_t su = d3 ? static_cast<size_t>(Nx) * N1 : static_cast<size_t>(Nx);
    const int t = threadIdx.x, T = blockDim.x;
    const int n = tc * L;  // elements of one array in LDS
    float2* const tw = smem;
    float2* const A = smem + L;
    float2* const B = A + n;
    float2* const S = B + n;          // [NF][tc][L]
    float2* const acc = S + NF * n;   // [NF][tc][L]
    for (int i = t; i < L; i += T) tw[i] = tw_g[i];
    const FastDiv ftc(tc), fL(L);  // n < 2^21: the LDS holds the lines
    // global element of line c at position w; loads and stores run with the
    // line index fastest, so a wave touches neighbouring kx
    auto at = [&](int c, int w) { return base + c + static_cast<size_t>(w) * su; };
    auto gin = [&](const float2* __restrict__ src, float2* dst) {
        for (int i = t; i < n; i += T) {
            const int w = ftc.quo(i), c = i - w * tc;
            dst[c * L + w] = gload(src + at(c, w));
        }
    };
    auto gout = [&](const float2* src, float2* __restrict__ dst) {
        for (int i = t; i < n; i += T) {
            const int w = ftc.quo(i), c = i - w * tc;
            gstore(dst + at(c, w), src[c * L + w]);
        }
    };
    // line and position of LDS element i
    auto lw = [&](int i, int& c, int& w) {
        c = fL.quo(i);
        w = i - c * L;
    };
    auto ws = [&](int w) { return w < (L >> 1) ? w : w - L; };
    auto kxs = [&](int c) { const int kx = kx0 + c; return kx < (Nx >> 1) ? kx : kx - Nx; };
    auto kq = [&](int c, int w) { return d3 ? mode_q(p, kxs(c), kos, ws(w)) : mode_q(p, kxs(c), ws(w), 0); };

    if constexpr (MODE == MODE_FWD_STORE) {
        gin(bufs.in, A);
        __syncthreads();
        const float2* r = mr_transform(A, B, tw, my, -1, tc);
        gout(r, bufs.S[bufs.sel]);
        return;
    }
    if constexpr (MODE == MODE_INV_OUT) {
        gin(bufs.S[bufs.sel], A);
        __syncthreads();
        const float2* r = mr_transform(A, B, tw, my, 1, tc);
        gout(r, bufs.out);
        return;
    }

    const int nf = p.nf;
    for (int f = 0; f < nf; ++f) gin(bufs.S[f], S + f * n);
    __syncthreads();
    // Fourier value of source src at LDS element i (line i / L, position i % L)
    auto source = [&](int src, int i, const ModeQ& q) -> float2 {
        if constexpr (GEN) {
            if (src >= PSS_MAXF) {
                const DevInterm& I = p.interm[src - PSS_MAXF];
                float2 v = make_float2(0.f, 0.f);
                for (int j = 0; j < I.nsrc; ++j) v = cadd(v, cmul(eval_op<true>(I.op[j], q), S[I.src[j] * n + i]));
                return cmul(v, cinv_implicit(1.f, eval_op<true>(I.den, q)));
            }
        }
        return S[src * n + i];
    };

    if constexpr (MODE == MODE_INTERM_OUT) {
        for (int i = t; i < n; i += T) {
            int c, w;
            lw(i, c, w);
            A[i] = source(PSS_MAXF + bufs.sel, i, kq(c, w));
        }
        __syncthreads();
        const float2* r = mr_transform(A, B, tw, my, 1, tc);
        gout(r, bufs.out);
        return;
    }

    if constexpr (MODE == MODE_STEP) {
        const uint32_t step = static_cast<uint32_t>(gload_u64(step_ctr)) + static_cast<uint32_t>(step_off);
        for (int i = t; i < nf * n; i += T) acc[i] = make_float2(0.f, 0.f);
        // channels: forward transforms of the products, M(q) per mode
        for (int ch = 0; ch < p.nch; ++ch) {
            const DevChannel& C = p.ch[ch];
            gin(bufs.N[ch], A);
            __syncthreads();
            const float2* r = mr_transform(A, B, tw, my, -1, tc);
            for (int i = t; i < n; i += T) {
                int c, w;
                lw(i, c, w);
                const ModeQ q = kq(c, w);
                for (int o = 0; o < C.nout; ++o) {
                    float2& d = acc[C.target[o] * n + i];
                    d = cadd(d, cmul(eval_op<GEN>(C.op[o], q), r[i]));
                }
            }
            __syncthreads();
        }
        // linear explicit terms, then the semi-implicit update with the noise
        for (int i = t; i < n && p.nd > 0; i += T) {
            int c, w;
            lw(i, c, w);
            const ModeQ q = kq(c, w);
            for (int d = 0; d < p.nd; ++d) {
                const DevDirect& Dd = p.direct[d];
                float2& a = acc[Dd.target * n + i];
                a = cadd(a, cmul(eval_op<GEN>(Dd.op, q), source(Dd.src, i, q)));
            }
        }
        __syncthreads();
        uint32_t bad = 0;
        for (int i = t; i < n; i += T) {
            int c, w;
            lw(i, c, w);
            const int kx = kx0 + c;
            const ModeQ q = kq(c, w);
            const uint32_t lin = static_cast<uint32_t>(at(c, w));
            // the linear index of the mode -k (each index modulo its size)
            const size_t wn = w ? L - w : 0;
            const size_t neg_line = d3 ? wn * N1 + static_cast<size_t>(ko ? N1 - ko : 0) : wn;
            const uint32_t lneg = static_cast<uint32_t>(neg_line * Nx + static_cast<size_t>(kx ? Nx - kx : 0));
            for (int f = 0; f < nf; ++f) {
                float2 r = cadd(S[f * n + i], cscale(acc[f * n + i], p.dt));
                if (p.noisy[f] != 0) r = cadd(r, noise_mode<GEN>(p, f, step, lin, lneg, q));
                r = cmul(r, cinv_implicit(p.dt, eval_op<GEN>(p.implicit_op[f], q)));
                S[f * n + i] = r;
                if (!(__builtin_isfinite(r.x) && __builtin_isfinite(r.y))) bad |= 1u << f;
            }
        }
        if (bad) atomicOr(flag, bad);
        __syncthreads();
        for (int f = 0; f < nf; ++f) gout(S + f * n, bufs.S[f]);
    }

    // MODE_STEP and MODE_PROLOGUE: inverse transforms of the de-aliased
    // factors from the (new) state
    for (int g = 0; g < p.ng; ++g) {
        const DevMask& mk = p.mask[g];
        for (int i = t; i < n; i += T) {
            int c, w;
            lw(i, c, w);
            A[i] = (d3 ? mask_keep(mk, kxs(c), kos, ws(w)) : mask_keep(mk, kxs(c), ws(w), 0))
                       ? source(p.gfield[g], i, kq(c, w))
                       : make_float2(0.f, 0.f);
        }
        __syncthreads();
        const float2* r = mr_transform(A, B, tw, my, 1, tc);
        gout(r, bufs.V[g]);
        __syncthreads();
    }
}

template <int MODE>
__global__ void __launch_bounds__(256)
    mr2_row_kernel(const DevPlan* __restrict__ plan, Bufs bufs, const float2* __restrict__ tw_g, MrPlan mx,
                   int64_t advance, uint64_t* __restrict__ step_ctr) {
    extern __shared__ float2 smem[];
    const DevPlan& p = *plan;
    const int Nx = mx.n;
    const size_t row = static_cast<size_t>(blockIdx.x) * Nx;
    const int t = threadIdx.x, T = blockDim.x;
    float2* const tw = smem;
    float2* const A = smem + Nx;
    float2* const B = smem + 2 * Nx;
    float* const u = reinterpret_cast<float*>(smem + 3 * Nx);  // [ng][Nx]
    for (int i = t; i < Nx; i += T) tw[i] = tw_g[i];

    if constexpr (MODE == MODE_R2C_IN) {
        for (int x = t; x < Nx; x += T) A[x] = make_float2(bufs.real_in[row + x], 0.f);
        __syncthreads();
        const float2* r = mr_transform(A, B, tw, mx, -1);
        for (int k = t; k < Nx; k += T) gstore(bufs.out + row + k, r[k]);
        return;
    }
    if constexpr (MODE == MODE_C2R_OUT) {
        for (int k = t; k < Nx; k += T) A[k] = gload(bufs.in + row + k);
        __syncthreads();
        const float2* r = mr_transform(A, B, tw, mx, 1);
        for (int x = t; x < Nx; x += T) bufs.real_out[row + x] = r[x].x * p.inv_n;
        return;
    }
    // MODE_STEP: factors to real space, products, forward x transforms
    for (int g = 0; g < p.ng; ++g) {
        for (int k = t; k < Nx; k += T) A[k] = gload(bufs.V[g] + row + k);
        __syncthreads();
        const float2* r = mr_transform(A, B, tw, mx, 1);
        for (int x = t; x < Nx; x += T) u[g * Nx + x] = r[x].x * p.inv_n;
        __syncthreads();
    }
    for (int ch = 0; ch < p.nch; ++ch) {
        const DevChannel& C = p.ch[ch];
        for (int x = t; x < Nx; x += T) {
            float w = 0.f;
            for (int k = 0; k < C.nprod; ++k) {
                const DevProd& pd = C.prod[k];
                float a = pd.coef;
                for (int g = 0; g < p.ng; ++g)
                    for (int e = 0; e < pd.pow[g]; ++e) a *= u[g * Nx + x];
                w += a;
            }
            A[x] = make_float2(w, 0.f);
        }
        __syncthreads();
        const float2* r = mr_transform(A, B, tw, mx, -1);
        for (int k = t; k < Nx; k += T) gstore(bufs.N[ch] + row + k, r[k]);
        __syncthreads();
    }
    if (advance != 0 && blockIdx.x == 0 && t == 0) *step_ctr += static_cast<uint64_t>(advance);
}

// 3D: transforms along y of the arrays of ya (in place allowed: a line is
// read whole before it is written), one block per (kx, z) line
__global__ void __launch_bounds__(256)
    mr3_ypass_kernel(const DevPlan* __restrict__ plan, YArgs ya, const float2* __restrict__ tw_g, MrPlan my, int sign,
                     int tc) {
    extern __shared__ float2 smem[];
    const DevPlan& p = *plan;
    const int Nx = p.n[0], Ny = my.n;
    const int nxb = Nx / tc;
    const int blk = xcd_block(blockIdx.x, gridDim.x);  // as in the column kernel
    const int kx0 = (blk % nxb) * tc, z = blk / nxb;
    const size_t base = static_cast<size_t>(z) * Nx * Ny + kx0;
    const int t = threadIdx.x, T = blockDim.x;
    const int n = tc * Ny;
    const FastDiv ftc(tc);
    float2* const tw = smem;
    float2* const A = smem + Ny;
    float2* const B = A + n;
    for (int i = t; i < Ny; i += T) tw[i] = tw_g[i];
    for (int a = 0; a < ya.n; ++a) {
        for (int i = t; i < n; i += T) {
            const int y = ftc.quo(i), c = i - y * tc;
            A[c * Ny + y] = gload(ya.src[a] + base + c + static_cast<size_t>(y) * Nx);
        }
        __syncthreads();
        const float2* r = mr_transform(A, B, tw, my, sign, tc);
        for (int i = t; i < n; i += T) {
            const int y = ftc.quo(i), c = i - y * tc;
            gstore(ya.dst[a] + base + c + static_cast<size_t>(y) * Nx, r[c * Ny + y]);
        }
        __syncthreads();
    }
}

hipError_t launch_mr3_ypass(int sign, const YArgs& ya, const LaunchArgs& a) {
    MrPlan my{};
    if (!mr_plan(a.ny, &my) || a.dim != 3) return hipErrorInvalidValue;
    if (ya.n <= 0) return hipSuccess;
    const int tc = a.geo.py;  // neighbouring y lines per block
    if (tc < 1 || a.nx % tc != 0) return hipErrorInvalidValue;
    const size_t lds = mr3_ypass_lds_bytes(my.n, tc);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    hipLaunchKernelGGL(mr3_ypass_kernel, dim3((a.nx / tc) * a.nz), dim3(256), lds, a.stream, a.plan, ya, a.tw_y, my,
                       sign, tc);
    return hipGetLastError();
}

hipError_t launch_mr2_col(int mode, int nf, const LaunchArgs& a) {
    MrPlan my{};
    if (!mr_plan(a.dim == 3 ? a.nz : a.ny, &my)) return hipErrorInvalidValue;
    const int NF = nf <= 1 ? 1 : (nf == 2 ? 2 : 4);
    const int tc = a.geo.tc;  // neighbouring lines per block
    if (tc < 1 || a.nx % tc != 0) return hipErrorInvalidValue;
    const size_t lds = mr2_col_lds_bytes(my.n, NF, tc);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    const dim3 grid((a.nx / tc) * (a.dim == 3 ? a.ny : 1)), block(256);
    const bool gen = a.general || mode == MODE_INTERM_OUT;
#define PSS_C2(NFV, G, M)                                                                                    \
    hipLaunchKernelGGL((mr2_col_kernel<NFV, G, M>), grid, block, lds, a.stream, a.plan, a.bufs, a.step_ctr,  \
                       a.flag, a.step_off, a.tw_u, my, tc)
#define PSS_C2F(M)                       \
    do {                                 \
        if (NF == 1) {                   \
            if (gen)                     \
                PSS_C2(1, true, M);      \
            else                         \
                PSS_C2(1, false, M);     \
        } else if (NF == 2) {            \
            if (gen)                     \
                PSS_C2(2, true, M);      \
            else                         \
                PSS_C2(2, false, M);     \
        } else {                         \
            if (gen)                     \
                PSS_C2(4, true, M);      \
            else                         \
                PSS_C2(4, false, M);     \
        }                                \
    } while (0)
    switch (mode) {
        case MODE_STEP: PSS_C2F(MODE_STEP); break;
        case MODE_PROLOGUE: PSS_C2F(MODE_PROLOGUE); break;
        case MODE_INTERM_OUT: PSS_C2F(MODE_INTERM_OUT); break;
        case MODE_FWD_STORE: PSS_C2(1, false, MODE_FWD_STORE); break;
        case MODE_INV_OUT: PSS_C2(1, false, MODE_INV_OUT); break;
        default: return hipErrorInvalidValue;
    }
#undef PSS_C2F
#undef PSS_C2
    return hipGetLastError();
}

hipError_t launch_mr2_row(int mode, const LaunchArgs& a) {
    MrPlan mx{};
    if (!mr_plan(a.nx, &mx)) return hipErrorInvalidValue;
    const size_t lds = mr2_row_lds_bytes(mx.n, a.ng);
    if (lds > 160 * 1024) return hipErrorInvalidValue;
    const dim3 grid(a.ny * (a.dim == 3 ? a.nz : 1)), block(256);
    uint64_t* ctr = const_cast<uint64_t*>(a.step_ctr);
    switch (mode) {
        case MODE_STEP:
            hipLaunchKernelGGL(mr2_row_kernel<MODE_STEP>, grid, block, lds, a.stream, a.plan, a.bufs, a.tw_x, mx,
                               a.advance, ctr);
            break;
        case MODE_R2C_IN:
            hipLaunchKernelGGL(mr2_row_kernel<MODE_R2C_IN>, grid, block, lds, a.stream, a.plan, a.bufs, a.tw_x, mx,
                               int64_t{0}, ctr);
            break;
        case MODE_C2R_OUT:
            hipLaunchKernelGGL(mr2_row_kernel<MODE_C2R_OUT>, grid, block, lds, a.stream, a.plan, a.bufs, a.tw_x, mx,
                               int64_t{0}, ctr);
            break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t mr2_setup() {
    const int lds = 160 * 1024;
#define PSS_C2A(NFV, G, M)                                                                                     \
    if (hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&mr2_col_kernel<NFV, G, M>),          \
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds))                   \
        return e;
#define PSS_C2B(M) PSS_C2A(1, false, M) PSS_C2A(1, true, M) PSS_C2A(2, false, M) PSS_C2A(2, true, M) \
    PSS_C2A(4, false, M) PSS_C2A(4, true, M)
    PSS_C2B(MODE_STEP)
    PSS_C2B(MODE_PROLOGUE)
    PSS_C2B(MODE_INTERM_OUT)
    PSS_C2A(1, false, MODE_FWD_STORE)
    PSS_C2A(1, false, MODE_INV_OUT)
#undef PSS_C2B
#undef PSS_C2A
#define PSS_R2A(M)                                                                                             \
    if (hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&mr2_row_kernel<M>),                  \
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds))                   \
        return e;
    PSS_R2A(MODE_STEP)
    PSS_R2A(MODE_R2C_IN)
    PSS_R2A(MODE_C2R_OUT)
#undef PSS_R2A
    return hipFuncSetAttribute(reinterpret_cast<const void*>(&mr3_ypass_kernel),
                               hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}
#endif  // PSS_COMMON

// ------------------------------------------------------- launch dispatch
// -------------------------------------------------------------- 1D lattices
// One block holds the whole line of N sites: T = N/4 threads, 4 modes each.
// A field's state is its full complex spectrum (Hermitian up to rounding) in
// natural mode order; thread t keeps modes k = D(t) + m T, the order in which
// the forward transform leaves them and the inverse transform takes them, so
// a step needs no reordering.  Real space is the real part of the inverse
// transform (as for every dimension).  A launch first forms the explicit
// contributions of its first step from the state, then takes its steps in
// registers, following the per-step list after eq:timeupdate: intermediate
// and de-aliased factors from the state, inverse transforms, products,
// forward transforms, noise, semi-implicit update.
template <int N, int NF, bool GEN, int MODE>
__global__ void __launch_bounds__(N / 4 < 64 ? 64 : N / 4)
    line1d_kernel(const DevPlan* __restrict__ plan, Bufs bufs, uint64_t* __restrict__ step_ctr,
                  uint32_t* __restrict__ flag, int nsteps, int advance, const float2* __restrict__ tw_g) {
    constexpr int P = 4;
    using FFT = LineFFT<N, P>;
    constexpr int T = FFT::T;
    extern __shared__ float2 smem[];
    const DevPlan& p = *plan;
    const int t = threadIdx.x;
    LdsLine ld;
    ld.wl = smem;
    ld.blk0 = smem + FFT::kReg;
    ld.blk1 = smem + 2 * FFT::kReg;
    ld.par = 0;
    float2* const twl = smem + FFT::kLds;
    float* const xst = reinterpret_cast<float*>(twl + N);  // real-space staging of the frames
    for (int i = t; i < N; i += T) twl[i] = tw_g[i];
    __syncthreads();
    const float2* tw = twl;
    const int dr = FFT::drev(t);
    // the modes of this thread: index k = dr + m T, signed kx, q, linear indices
    ModeQ q[P];
    float q2[P];
    uint32_t lin[P], lneg[P];
#pragma unroll
    for (int m = 0; m < P; ++m) {
        const int k = dr + m * T;
        q[m] = mode_q(p, k < (N >> 1) ? k : k - N, 0, 0);
        q2[m] = q[m].q2;
        lin[m] = static_cast<uint32_t>(k);
        lneg[m] = static_cast<uint32_t>((N - k) & (N - 1));
    }

    if constexpr (MODE == MODE_FWD_STORE) {
        float2 v[P];
#pragma unroll
        for (int m = 0; m < P; ++m) v[m] = make_float2(bufs.real_in[t + m * T], 0.f);
        FFT::template dif<-1>(v, ld, t, tw);
#pragma unroll
        for (int m = 0; m < P; ++m) gstore(bufs.S[bufs.sel] + dr + m * T, v[m]);
        return;
    }
    if constexpr (MODE == MODE_INV_OUT) {
        float2 v[P];
#pragma unroll
        for (int m = 0; m < P; ++m) v[m] = gload(bufs.S[bufs.sel] + dr + m * T);
        FFT::template dit<1>(v, ld, t, tw);
#pragma unroll
        for (int m = 0; m < P; ++m) bufs.real_out[t + m * T] = v[m].x * p.inv_n;
        return;
    }

    float2 s[NF][P];
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int m = 0; m < P; ++m) s[f][m] = f < p.nf ? gload(bufs.S[f] + dr + m * T) : make_float2(0.f, 0.f);

    // the Fourier values of source `src` (a dynamic field, or an intermediate
    // psi = sum_k op_k phi_k / (1 - L_psi)) at this thread's modes
    auto source = [&](int src, float2 (&v)[P]) {
        if constexpr (GEN) {
            if (src >= PSS_MAXF) {
                const DevInterm& I = p.interm[src - PSS_MAXF];
#pragma unroll
                for (int m = 0; m < P; ++m) v[m] = make_float2(0.f, 0.f);
                for (int k = 0; k < I.nsrc; ++k) {
                    const int sk = I.src[k];
#pragma unroll
                    for (int m = 0; m < P; ++m) v[m] = cadd(v[m], cmul(eval_op<true>(I.op[k], q[m]), pick(s, sk, m)));
                }
#pragma unroll
                for (int m = 0; m < P; ++m) v[m] = cmul(v[m], cinv_implicit(1.f, eval_op<true>(I.den, q[m])));
                return;
            }
        }
#pragma unroll
        for (int m = 0; m < P; ++m) v[m] = pick(s, src, m);
    };

    if constexpr (MODE == MODE_INTERM_OUT) {
        float2 v[P];
        source(PSS_MAXF + bufs.sel, v);
        FFT::template dit<1>(v, ld, t, tw);
#pragma unroll
        for (int m = 0; m < P; ++m) bufs.real_out[t + m * T] = v[m].x * p.inv_n;
        return;
    }

    // MODE_STEP.  acc: the explicit contributions sum_ch M_ch(q) F[products]
    float2 acc[NF][P];
    auto channels = [&]() {
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int m = 0; m < P; ++m) acc[f][m] = make_float2(0.f, 0.f);
        if (p.nch == 0) return;
        // real-space values of the de-aliased factors at x = t + m T
        float u[PSS_MAXG][P];
#pragma unroll
        for (int g = 0; g < PSS_MAXG; ++g) {
            if (g >= p.ng) break;
            const DevMask& mk = p.mask[g];
            float2 v[P];
            source(p.gfield[g], v);
#pragma unroll
            for (int m = 0; m < P; ++m) {
                const int k = dr + m * T;
                if (!mask_keep(mk, k < (N >> 1) ? k : k - N, 0, 0)) v[m] = make_float2(0.f, 0.f);
            }
            FFT::template dit<1>(v, ld, t, tw);
#pragma unroll
            for (int m = 0; m < P; ++m) u[g][m] = v[m].x * p.inv_n;
        }
        for (int ch = 0; ch < p.nch; ++ch) {
            const DevChannel& C = p.ch[ch];
            float2 w[P];
#pragma unroll
            for (int m = 0; m < P; ++m) w[m] = make_float2(0.f, 0.f);
            for (int k = 0; k < C.nprod; ++k) {
                const DevProd& pd = C.prod[k];
                uint64_t pw;
                __builtin_memcpy(&pw, pd.pow, sizeof(pw));
#pragma unroll
                for (int m = 0; m < P; ++m) {
                    float a = pd.coef;
#pragma unroll
                    for (int g = 0; g < PSS_MAXG; ++g) {
                        if (g >= p.ng) break;
                        const int pg = static_cast<int>((pw >> (8 * g)) & 0xffull);
                        for (int e = 0; e < pg; ++e) a *= u[g][m];
                    }
                    w[m].x += a;
                }
            }
            FFT::template dif<-1>(w, ld, t, tw);
            for (int o = 0; o < C.nout; ++o)
#pragma unroll
                for (int m = 0; m < P; ++m) add_to(acc, C.target[o], m, cmul(eval_op<GEN>(C.op[o], q[m]), w[m]));
        }
    };

    const uint32_t step0 = static_cast<uint32_t>(gload_u64(step_ctr));
    uint32_t bad = 0;
    channels();
    for (int sn = 0; sn < nsteps; ++sn) {
        const uint32_t step = step0 + static_cast<uint32_t>(sn);
        // linear explicit terms from the step-n state
        for (int d = 0; d < p.nd; ++d) {
            const DevDirect& Dd = p.direct[d];
            float2 src[P];
            source(Dd.src, src);
#pragma unroll
            for (int m = 0; m < P; ++m) add_to(acc, Dd.target, m, cmul(eval_op<GEN>(Dd.op, q[m]), src[m]));
        }
        // semi-implicit update with the noise of this step
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            if (f >= p.nf) continue;
            const bool noisy = p.noisy[f] != 0;
#pragma unroll
            for (int m = 0; m < P; ++m) {
                float2 r = cadd(s[f][m], cscale(acc[f][m], p.dt));
                if (noisy) r = cadd(r, noise_mode<GEN>(p, f, step, lin[m], lneg[m], q[m]));
                s[f][m] = cmul(r, cinv_implicit(p.dt, eval_op<GEN>(p.implicit_op[f], q[m])));
            }
        }
        // boundary frames: the new state's real space takes the frame values
        // on the frame sites (staged through LDS), then is transformed back
#pragma unroll
        for (int f = 0; f < NF; ++f) {
            if (f >= p.nf || p.nframe[f] == 0) continue;
            float2 v[P];
#pragma unroll
            for (int m = 0; m < P; ++m) v[m] = s[f][m];
            FFT::template dit<1>(v, ld, t, tw);
#pragma unroll
            for (int m = 0; m < P; ++m) xst[t + m * T] = v[m].x * p.inv_n;
            __syncthreads();
            const int2* __restrict__ fr = p.frame[f];
            for (int i = t; i < p.nframe[f]; i += T) {
                const int2 e = fr[i];
                xst[e.x] = __int_as_float(e.y);
            }
            __syncthreads();
#pragma unroll
            for (int m = 0; m < P; ++m) v[m] = make_float2(xst[t + m * T], 0.f);
            __syncthreads();  // the staging line is free again
            FFT::template dif<-1>(v, ld, t, tw);
#pragma unroll
            for (int m = 0; m < P; ++m) s[f][m] = v[m];
        }
#pragma unroll
        for (int f = 0; f < NF; ++f)
            if (f < p.nf)
#pragma unroll
                for (int m = 0; m < P; ++m)
                    if (!(__builtin_isfinite(s[f][m].x) && __builtin_isfinite(s[f][m].y))) bad |= 1u << f;
        if (sn + 1 < nsteps) channels();  // the next launch forms its first step's anew
    }
#pragma unroll
    for (int f = 0; f < NF; ++f)
        if (f < p.nf)
#pragma unroll
            for (int m = 0; m < P; ++m) gstore(bufs.S[f] + dr + m * T, s[f][m]);
    if (bad) atomicOr(flag, bad);
    __syncthreads();  // every thread has read the counter
    if (advance && t == 0) *step_ctr += static_cast<uint64_t>(nsteps);
}

// This file is compiled once per line length with -DPSS_LINE_LEN=<L> (the
// kernels of that length) and once with -DPSS_COMMON (utilities and the
// length dispatch), so the instantiations build in parallel.
#if defined(PSS_LINE_LEN)
template <int L, int P, int NF, int DIM, bool TABLE>
static hipError_t launch_update_tab(int mode, const LaunchArgs& a, dim3 grid, dim3 block, size_t lds) {
#define PSS_UPD(M, G, NFV)                                                                                        \
    hipLaunchKernelGGL((update_kernel<L, P, NFV, M, DIM, G, TABLE>), grid, block, lds, a.stream, a.members, a.plans, \
                       a.plan, a.bufs, a.geo, a.step_ctr, a.flag, a.step_off, a.tw_u)
    switch (mode) {
        case MODE_STEP:
            if (a.general)
                PSS_UPD(MODE_STEP, true, NF);
            else
                PSS_UPD(MODE_STEP, false, NF);
            break;
        case MODE_PROLOGUE:
            if (a.general)
                PSS_UPD(MODE_PROLOGUE, true, NF);
            else
                PSS_UPD(MODE_PROLOGUE, false, NF);
            break;
        case MODE_INTERM_OUT: PSS_UPD(MODE_INTERM_OUT, true, NF); break;
        default: return hipErrorInvalidValue;
    }
#undef PSS_UPD
    return hipGetLastError();
}

template <int L, int P, int NF, int DIM>
static hipError_t launch_update_d(int mode, const LaunchArgs& a) {
    const int threads = a.geo.tc * a.geo.to * (L / P);
    const size_t lds = update_lds_bytes(L, P, a.geo.tc, a.geo.to);
    const bool tab = mode == MODE_STEP || mode == MODE_PROLOGUE || mode == MODE_INTERM_OUT;
    if (tab && (!a.members || !a.plans || a.nmem < 1)) return hipErrorInvalidValue;
    if (mode == MODE_INTERM_OUT && a.nmem != 1) return hipErrorInvalidValue;
    dim3 grid(a.geo.nublk, tab ? a.nmem : 1), block(threads);
    if (tab) {
        // one lattice: buffers, counter and flag come from the arguments
        if (a.nmem > 1) return launch_update_tab<L, P, NF, DIM, true>(mode, a, grid, block, lds);
        return launch_update_tab<L, P, NF, DIM, false>(mode, a, grid, block, lds);
    }
    switch (mode) {
        case MODE_FWD_STORE:
            hipLaunchKernelGGL((update_kernel<L, P, 1, MODE_FWD_STORE, DIM, false, false>), grid, block, lds, a.stream,
                               a.members, a.plans, a.plan, a.bufs, a.geo, a.step_ctr, a.flag, a.step_off, a.tw_u);
            break;
        case MODE_INV_OUT:
            hipLaunchKernelGGL((update_kernel<L, P, 1, MODE_INV_OUT, DIM, false, false>), grid, block, lds, a.stream,
                               a.members, a.plans, a.plan, a.bufs, a.geo, a.step_ctr, a.flag, a.step_off, a.tw_u);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int L, int P, int NF>
static hipError_t launch_update_t(int mode, const LaunchArgs& a) {
    return a.dim == 3 ? launch_update_d<L, P, NF, 3>(mode, a) : launch_update_d<L, P, NF, 2>(mode, a);
}

template <int L, int P, int NG>
static hipError_t launch_xrow_t(int mode, const LaunchArgs& a) {
    const int threads = (a.geo.rb / 2) * (L / P);
    const size_t lds = xrow_lds_bytes(L, P, a.geo.rb);
    const bool tab = mode == MODE_STEP;
    if (tab && (!a.members || !a.plans || a.nmem < 1)) return hipErrorInvalidValue;
    dim3 grid(a.geo.nrowblk, tab ? a.nmem : 1), block(threads);
    uint64_t* ctr = const_cast<uint64_t*>(a.step_ctr);
    switch (mode) {
        case MODE_STEP:
            if (a.nmem > 1)
                hipLaunchKernelGGL((xrow_kernel<L, P, NG, MODE_STEP, true>), grid, block, lds, a.stream, a.members,
                                   a.plans, a.plan, a.bufs, a.geo, a.tw_x, a.advance, ctr);
            else
                hipLaunchKernelGGL((xrow_kernel<L, P, NG, MODE_STEP, false>), grid, block, lds, a.stream, a.members,
                                   a.plans, a.plan, a.bufs, a.geo, a.tw_x, a.advance, ctr);
            break;
        case MODE_R2C_IN:
            hipLaunchKernelGGL((xrow_kernel<L, P, 1, MODE_R2C_IN, false>), grid, block, lds, a.stream, a.members,
                               a.plans, a.plan, a.bufs, a.geo, a.tw_x, int64_t{0}, ctr);
            break;
        case MODE_C2R_OUT:
            hipLaunchKernelGGL((xrow_kernel<L, P, 1, MODE_C2R_OUT, false>), grid, block, lds, a.stream, a.members,
                               a.plans, a.plan, a.bufs, a.geo, a.tw_x, int64_t{0}, ctr);
            break;
        case MODE_ADJROW:
            if ((threads & 63) != 0 && threads > 64) return hipErrorInvalidValue;  // block_sum_to_slot's shapes
            if constexpr (NG == 2) {
                hipLaunchKernelGGL((xrow_kernel<L, P, 2, MODE_ADJROW, false>), grid, block, lds, a.stream, a.members,
                                   a.plans, a.plan, a.bufs, a.geo, a.tw_x, int64_t{0}, ctr);
                break;
            }
            return hipErrorInvalidValue;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

#define PSS_CAT2(a, b) a##b
#define PSS_CAT(a, b) PSS_CAT2(a, b)

// points-per-thread variants: P = geo.pu (update) or geo.px (x kernel), any
// of 16, 8, 4 not above the cap for the number of register arrays
template <int L, int CAP, class F>
static hipError_t with_points(int want, F&& f) {
    if constexpr (L >= 16 && CAP >= 16) {
        if (want == 16) return f(std::integral_constant<int, 16>{});
    }
    if constexpr (L >= 8 && CAP >= 8) {
        if (want == 8) return f(std::integral_constant<int, 8>{});
    }
    if constexpr (L >= 4 && CAP >= 4) {
        if (want == 4) return f(std::integral_constant<int, 4>{});
    }
    if constexpr (L < 4) {
        if (want == L) return f(std::integral_constant<int, L>{});
    }
    return hipErrorInvalidValue;
}

template <int NF, bool GEN>
static hipError_t launch_line1d_t(int mode, const LaunchArgs& a) {
    constexpr int N = PSS_LINE_LEN;
    const dim3 grid(1), block(N / 4);
    const size_t lds = line1d_lds_bytes(N);
    uint64_t* ctr = const_cast<uint64_t*>(a.step_ctr);
#define PSS_L1(M)                                                                                                 \
    hipLaunchKernelGGL((line1d_kernel<N, NF, GEN, M>), grid, block, lds, a.stream, a.plan, a.bufs, ctr, a.flag, \
                       a.nsteps, a.advance != 0 ? 1 : 0, a.tw_x)
    switch (mode) {
        case MODE_STEP: PSS_L1(MODE_STEP); break;
        case MODE_FWD_STORE: PSS_L1(MODE_FWD_STORE); break;
        case MODE_INV_OUT: PSS_L1(MODE_INV_OUT); break;
        case MODE_INTERM_OUT: PSS_L1(MODE_INTERM_OUT); break;
        default: return hipErrorInvalidValue;
    }
#undef PSS_L1
    return hipGetLastError();
}

hipError_t PSS_CAT(launch_line1d_L, PSS_LINE_LEN)(int mode, int nf, const LaunchArgs& a) {
    if (mode == MODE_FWD_STORE || mode == MODE_INV_OUT) return launch_line1d_t<1, false>(mode, a);
    const bool gen = a.general || mode == MODE_INTERM_OUT;
    if (nf <= 1) return gen ? launch_line1d_t<1, true>(mode, a) : launch_line1d_t<1, false>(mode, a);
    if (nf == 2) return gen ? launch_line1d_t<2, true>(mode, a) : launch_line1d_t<2, false>(mode, a);
    if (nf <= 4) return gen ? launch_line1d_t<4, true>(mode, a) : launch_line1d_t<4, false>(mode, a);
    return hipErrorInvalidValue;
}

hipError_t PSS_CAT(line1d_setup_L, PSS_LINE_LEN)() {
    constexpr int N = PSS_LINE_LEN;
    const int lds = static_cast<int>(line1d_lds_bytes(N));
#define PSS_L1A(NFV, G, M)                                                                                       \
    if (hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&line1d_kernel<N, NFV, G, M>),          \
                                           hipFuncAttributeMaxDynamicSharedMemorySize, lds))                     \
        return e;
#define PSS_L1B(M) PSS_L1A(1, false, M) PSS_L1A(1, true, M) PSS_L1A(2, false, M) PSS_L1A(2, true, M) \
    PSS_L1A(4, false, M) PSS_L1A(4, true, M)
    PSS_L1B(MODE_STEP)
    PSS_L1B(MODE_INTERM_OUT)
    PSS_L1A(1, false, MODE_FWD_STORE)
    PSS_L1A(1, false, MODE_INV_OUT)
#undef PSS_L1B
#undef PSS_L1A
    return hipSuccess;
}

hipError_t PSS_CAT(launch_update_L, PSS_LINE_LEN)(int mode, int nf, const LaunchArgs& a) {
    constexpr int L = PSS_LINE_LEN;
    const int pu = a.geo.pu;
    if (mode == MODE_FWD_STORE || mode == MODE_INV_OUT || nf <= 1)
        return with_points<L, 16>(pu, [&](auto P) { return launch_update_t<L, decltype(P)::value, 1>(mode, a); });
    if (nf == 2)
        return with_points<L, 8>(pu, [&](auto P) { return launch_update_t<L, decltype(P)::value, 2>(mode, a); });
    if (nf <= 4)
        return with_points<L, 4>(pu, [&](auto P) { return launch_update_t<L, decltype(P)::value, 4>(mode, a); });
    return hipErrorInvalidValue;
}

hipError_t PSS_CAT(launch_ypass_L, PSS_LINE_LEN)(int mode, const YArgs& ya, const LaunchArgs& a) {
    constexpr int L = PSS_LINE_LEN;
    return with_points<L, 16>(a.geo.py, [&](auto PP) {
        constexpr int P = decltype(PP)::value;
        const int threads = a.geo.tc * a.geo.tz * (L / P);
        const size_t lds = ypass_lds_bytes(L, P, a.geo.tc, a.geo.tz);
        dim3 grid(a.geo.nyblk), block(threads);
        if (mode == MODE_YINV) {
            hipLaunchKernelGGL((ypass_kernel<L, P, MODE_YINV>), grid, block, lds, a.stream, ya, a.geo, a.tw_y);
        } else if (mode == MODE_YFWD) {
            hipLaunchKernelGGL((ypass_kernel<L, P, MODE_YFWD>), grid, block, lds, a.stream, ya, a.geo, a.tw_y);
        } else {
            return hipErrorInvalidValue;
        }
        return hipGetLastError();
    });
}

hipError_t PSS_CAT(launch_adjcol_L, PSS_LINE_LEN)(int mode, const AdjArgs& aa, const LaunchArgs& a) {
    constexpr int L = PSS_LINE_LEN;
    return with_points<L, 16>(a.geo.pu, [&](auto PP) {
        constexpr int P = decltype(PP)::value;
        const int threads = a.geo.tc * (L / P);
        const size_t lds = update_lds_bytes(L, P, a.geo.tc, 1);
        dim3 grid(a.geo.nublk), block(threads);
        if (a.dim != 2 || a.geo.to != 1) return hipErrorInvalidValue;
        if ((threads & 63) != 0 && threads > 64) return hipErrorInvalidValue;  // block_sum_to_slot's shapes
        if (mode == MODE_ADJCOL) {
            hipLaunchKernelGGL((adjcol_kernel<L, P, MODE_ADJCOL>), grid, block, lds, a.stream, aa, a.geo, a.tw_u);
        } else if (mode == MODE_ADJFIN) {
            hipLaunchKernelGGL((adjcol_kernel<L, P, MODE_ADJFIN>), grid, block, lds, a.stream, aa, a.geo, a.tw_u);
        } else {
            return hipErrorInvalidValue;
        }
        return hipGetLastError();
    });
}

hipError_t PSS_CAT(launch_xrow_L, PSS_LINE_LEN)(int mode, int ng, const LaunchArgs& a) {
    constexpr int L = PSS_LINE_LEN;
    const int px = a.geo.px;
    if ((mode != MODE_STEP && mode != MODE_ADJROW) || ng <= 1)
        return with_points<L, 16>(px, [&](auto P) { return launch_xrow_t<L, decltype(P)::value, 1>(mode, a); });
    if (ng == 2)
        return with_points<L, 8>(px, [&](auto P) { return launch_xrow_t<L, decltype(P)::value, 2>(mode, a); });
    if (ng == 3)
        return with_points<L, 4>(px, [&](auto P) { return launch_xrow_t<L, decltype(P)::value, 3>(mode, a); });
    if (ng == 4)
        return with_points<L, 4>(px, [&](auto P) { return launch_xrow_t<L, decltype(P)::value, 4>(mode, a); });
    if (mode != MODE_STEP) return hipErrorInvalidValue;
    // five to eight factor slots (multi-field flow models): one variant with
    // room for eight, 4 points per thread
    if (ng <= PSS_MAXG)
        return with_points<L, 4>(px, [&](auto P) { return launch_xrow_t<L, decltype(P)::value, PSS_MAXG>(mode, a); });
    return hipErrorInvalidValue;
}
#endif  // PSS_LINE_LEN

#if defined(PSS_BATCH)
// ------------------------------------------------------ fused batch launches
// One launch per phase for a whole batch: block b (XCD-ordered) finds its
// class in the work list, then its member and tile, and runs the block body
// built for that class's line length.  The update launch uses unpadded
// transform exchanges: the pad's address arithmetic would raise the register
// count of a kernel that holds every line length's body, and with it cut the
// waves per SIMD from 4 to 3 (padding moves data only, never the results).
__device__ __forceinline__ int batch_class_of(const BatchLaunch& bl, int b) {
    int k = 0;
    for (int i = 1; i < bl.ncls; ++i)
        if (b >= bl.cls[i].start) k = i;
    return k;
}

__global__ void __launch_bounds__(256) batch_update_kernel(BatchLaunch bl) {
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const BatchClass& C = bl.cls[batch_class_of(bl, b)];
    const int rel = b - C.start;
    const int mi = rel / C.nblk;
    const int blk = rel - mi * C.nblk;
    const Bufs none{};
#define PSS_BU(LL)                                                                                                 \
    case LL:                                                                                                       \
        update_block<LL, 4, 1, MODE_STEP, 2, false, true, 0>(mi, blk, C.members, C.plans, nullptr, none, C.geo,       \
                                                             nullptr,                                                 \
                                                          nullptr, bl.step_off, C.tw);                             \
        break;
    switch (C.L) {
        PSS_BU(64)
        PSS_BU(128)
        PSS_BU(256)
        PSS_BU(512)
        PSS_BU(1024)
        default: break;
    }
#undef PSS_BU
}

__global__ void __launch_bounds__(256) batch_xrow_kernel(BatchLaunch bl) {
    const int b = xcd_block(blockIdx.x, gridDim.x);
    const BatchClass& C = bl.cls[batch_class_of(bl, b)];
    const int rel = b - C.start;
    const int mi = rel / C.nblk;
    const int blk = rel - mi * C.nblk;
    const Bufs none{};
#define PSS_BX(LL)                                                                                          \
    case LL:                                                                                                \
        xrow_block<LL, 4, 1, MODE_STEP, true>(mi, blk, C.members, C.plans, nullptr, none, C.geo, C.tw, bl.advance, \
                                              nullptr);                                                     \
        break;
    switch (C.L) {
        PSS_BX(64)
        PSS_BX(128)
        PSS_BX(256)
        PSS_BX(512)
        PSS_BX(1024)
        default: break;
    }
#undef PSS_BX
}

// ------------------------------------------------- LDS-resident multi-step
// One block holds a whole lattice: its state in registers (each thread keeps
// the slots of its column lines), the channel and factor arrays in one LDS
// array X[c][position] (column stride Ny + 1), which each phase overwrites in
// place: the column phase reads a column's channel values and writes its
// factor values, the row phase reads a row pair's factor values and writes
// its channel values.  The two phases are the update kernel's and the x
// kernel's line bodies with LDS in place of the packed-column arrays: the
// same transforms (4 points per thread; every line fits in a wave, so only
// the packed line's exchange and the phase changes take block barriers), the
// same operations in the same order, and the same position order of the
// exchanged arrays (the x phase works on positions as rows).  The launch
// loads the state and the channel array, runs rl.nsteps steps, stores both
// back and moves the member's step counter on.
template <int LX, int LY>
__global__ void __launch_bounds__(resident_threads(LX, LY)) resident_kernel(ResidentLaunch rl) {
    constexpr int P = 4;
    using FY = LineFFT<LY, P>;
    using FX = LineFFT<LX, P>;
    static_assert(!FY::kCross && !FX::kCross, "lines held by one wave");
    constexpr int TY = FY::T, TX = FX::T;
    constexpr int NC = LX / 2;                      // packed columns
    constexpr int NTHR = resident_threads(LX, LY);
    constexpr int CPR = NTHR / TY, RPR = NTHR / TX;  // column lines, row pairs per round
    constexpr int CR = NC / CPR;                     // rounds of each phase
    static_assert(CR * CPR == NC && CR * RPR == LY / 2, "whole rounds");
    constexpr int XS = LY + 1;                       // column stride of X
    constexpr int LPW = 64 / TY;                     // column lines per wave
    extern __shared__ float2 smem[];
    float2* const X = smem;
    float2* const scr = X + NC * XS;                 // one exchange region per line of a round
    constexpr int SCR = CPR * FY::kReg > RPR * FX::kReg ? CPR * FY::kReg : RPR * FX::kReg;
    float2* const xbuf = scr + SCR;                  // packed-line exchange (LY)
    float2* const twy = xbuf + LY;
    float2* const twx = twy + LY;
    const int mi = xcd_block(blockIdx.x, gridDim.x);
    const Member& mem = rl.members[mi];
    const DevPlan& p = rl.plans[mi];
    const int tid = threadIdx.x;
    const int tc = rl.geo.tc, lt = rl.geo.tc_log2;
    const int nx = p.n[0];
    float2* __restrict__ Sg = mem.bufs.S[0];
    float2* __restrict__ Ng = mem.bufs.N[0];

    for (int i = tid; i < LY; i += NTHR) twy[i] = rl.tw_y[i];
    for (int i = tid; i < LX; i += NTHR) twx[i] = rl.tw_x[i];
    // column phase: line li of the round, thread t of the line
    const int li = tid / TY, tcol = tid & (TY - 1);
    const int dry = FY::drev(tcol);
    LdsLine ldc;
    ldc.wl = scr + li * FY::kReg;
    ldc.blk0 = ldc.blk1 = nullptr;
    ldc.par = 0;
    // row phase: pair pi of the round, thread t of the pair
    const int pi = tid / TX, trow = tid & (TX - 1);
    const int drx = FX::drev(trow);
    LdsLine ldr;
    ldr.wl = scr + pi * FX::kReg;
    ldr.blk0 = ldr.blk1 = nullptr;
    ldr.par = 0;

    // the state of this thread's column slots, and the channel array
    float2 st[CR][P];
#pragma unroll
    for (int r = 0; r < CR; ++r) {
        const int c = r * CPR + li;
        const size_t base = (static_cast<size_t>(c >> lt) * LY << lt) + (c & (tc - 1));
#pragma unroll
        for (int m = 0; m < P; ++m) st[r][m] = gload(Sg + base + static_cast<size_t>(tcol + m * TY) * tc);
    }
    for (int i = tid; i < NC * LY; i += NTHR) {
        const int ct = i / (LY * tc), rem = i - ct * (LY * tc);
        const int y = rem >> lt, c = (ct << lt) + (rem & (tc - 1));
        X[c * XS + y] = gload(Ng + i);
    }
    const uint32_t step0 = static_cast<uint32_t>(gload_u64(mem.step_ctr));
    __syncthreads();

    uint32_t bad = 0;
    for (int sn = 0; sn < rl.nsteps; ++sn) {
        const uint32_t step = step0 + static_cast<uint32_t>(sn);
        // ---- column phase: forward y transform of the channel, update,
        // de-aliased inverse y transform of the factor
#pragma unroll
        for (int r = 0; r < CR; ++r) {
            const int c = r * CPR + li;
            const bool blk_packed = r == 0;  // the round holding column 0 (block-uniform)
            const bool packed = c == 0;
            const bool pair_lane = packed && tcol == 0;
            const int kx_l = c, ky_l = 0;
            float2* const col = X + c * XS;
            auto exchange = [&](float2 (&v)[P], bool forward) {
                if (!blk_packed) return;
                if (packed) {
#pragma unroll
                    for (int m = 0; m < P; ++m) xbuf[tcol + m * TY] = v[m];
                }
                __syncthreads();
                if (packed) {
#pragma unroll
                    for (int m = 0; m < P; ++m) {
                        const int u = tcol + m * TY;
                        const float2 b = xbuf[(LY - u) & (LY - 1)];
                        v[m] = forward ? to_slot<LY>(u, v[m], b) : from_slot<LY>(u, v[m], b);
                    }
                }
                __syncthreads();
            };
            const LineModes lmode = line_modes<LY, 2>(p, packed, kx_l, ky_l);
            float2(&s)[P] = st[r];
            float q2[P];
            uint32_t lin[P], lneg[P];
#pragma unroll
            for (int m = 0; m < P; ++m) slot_at<LY>(lmode, tcol + m * TY, q2[m], lin[m], lneg[m]);
            float2 acc[1][P];
#pragma unroll
            for (int m = 0; m < P; ++m) acc[0][m] = make_float2(0.f, 0.f);
            if (p.nch > 0) {
                const DevChannel& C = p.ch[0];
                float2 v[P];
#pragma unroll
                for (int m = 0; m < P; ++m) v[m] = col[tcol + m * TY];
                FY::template dit<-1>(v, ldc, tcol, twy);
                exchange(v, true);
                float M[P];
                horner_p(C.op[0], q2, M);
#pragma unroll
                for (int m = 0; m < P; ++m)
                    if (!(pair_lane && (m == 0 || m == P / 2))) add_to(acc, C.target[0], m, cscale(v[m], M[m]));
                if (pair_lane) pair_accumulate<2, false>(acc, C.target[0], v, p, C.op[0], ky_l, LY);
            }
            for (int d = 0; d < p.nd; ++d) {
                const DevDirect& Dd = p.direct[d];
                float2 src[P];
#pragma unroll
                for (int m = 0; m < P; ++m) src[m] = s[m];
                float M[P];
                horner_p(Dd.op, q2, M);
#pragma unroll
                for (int m = 0; m < P; ++m)
                    if (!(pair_lane && (m == 0 || m == P / 2))) add_to(acc, Dd.target, m, cscale(src[m], M[m]));
                if (pair_lane) pair_accumulate<2, false>(acc, Dd.target, src, p, Dd.op, ky_l, LY);
            }
            {
                const bool noisy = p.noisy[0] != 0;
                const float2 old0 = s[0], oldh = s[P / 2];
                float Ar[P], Dn[P];
                horner_p(p.implicit_op[0], q2, Ar);
                if (noisy) horner_p(p.noise_op[0], q2, Dn);
#pragma unroll
                for (int m = 0; m < P; ++m) {
                    float2 rr = cadd(s[m], cscale(acc[0][m], p.dt));
                    if (noisy) rr = cadd(rr, noise_value(p, 0, step, lin[m], lneg[m], Dn[m]));
                    s[m] = cscale(rr, __builtin_amdgcn_rcpf(fmaf(-p.dt, Ar[m], 1.f)));
                }
                if (pair_lane) {
                    s[0] = pair_update_d<2, false>(p, 0, step, ky_l, 0, LY, old0, acc[0][0], noisy);
                    s[P / 2] = pair_update_d<2, false>(p, 0, step, ky_l, LY >> 1, LY, oldh, acc[0][P / 2], noisy);
                }
                bool fin = true;
#pragma unroll
                for (int m = 0; m < P; ++m) fin = fin && __builtin_isfinite(s[m].x) && __builtin_isfinite(s[m].y);
                if (!fin) bad |= 1u;
            }
            // de-aliased inverse transform of the factor (lines of a wave whose
            // first column is past the kept ones are never read)
            if (p.ng > 0 && (c / LPW) * LPW < p.mask[0].ncol) {
                const DevMask& mk = p.mask[0];
                const int lim = line_lim<2>(mk, packed ? 0 : kx_l, ky_l, LY);
                const int limN = line_lim<2>(mk, -(nx >> 1), ky_l, LY);
                float2 v[P];
#pragma unroll
                for (int m = 0; m < P; ++m) {
                    const int u = tcol + m * TY;
                    const bool upper = packed && u > (LY >> 1);
                    const int w = packed ? (upper ? LY - u : u) : (u < (LY >> 1) ? u : u - LY);
                    v[m] = w * w <= (upper ? limN : lim) ? s[m] : make_float2(0.f, 0.f);
                }
                if (pair_lane) {
                    const int wh = (LY >> 1) * (LY >> 1);
                    const float2 a0 = s[0], ah = s[P / 2];
                    v[0] = make_float2(0 <= lim ? a0.x : 0.f, 0 <= limN ? a0.y : 0.f);
                    v[P / 2] = make_float2(wh <= lim ? ah.x : 0.f, wh <= limN ? ah.y : 0.f);
                }
                exchange(v, false);
                FY::template dif<1>(v, ldc, tcol, twy);
#pragma unroll
                for (int m = 0; m < P; ++m) col[tcol + m * TY] = v[m];
            } else if (blk_packed) {
                // the packed line's exchange barriers are block-wide
                __syncthreads();
                __syncthreads();
            }
        }
        __syncthreads();
        // ---- row phase: inverse x transform of each row pair's factor
        // values, the products, forward x transform into the channel values
#pragma unroll
        for (int r = 0; r < CR; ++r) {
            const int p0 = 2 * (r * RPR + pi);  // first position of the pair
            if (p.nch == 0) break;
            const int ncol = p.mask[0].ncol;
            float2 v[P];
            {
                float2 a[P], b[P];
#pragma unroll
                for (int m = 0; m < P; ++m) {
                    const int k = drx + m * TX;
                    const int kk = (k == NC) ? 0 : (k < NC ? k : LX - k);
                    const int kc = kk < ncol ? kk : 0;
                    a[m] = X[kc * XS + p0];
                    b[m] = X[kc * XS + p0 + 1];
                }
#pragma unroll
                for (int m = 0; m < P; ++m) {
                    const int k = drx + m * TX;
                    const int kk = (k == NC) ? 0 : (k < NC ? k : LX - k);
                    const float2 zero = make_float2(0.f, 0.f);
                    const float2 am = kk < ncol ? a[m] : zero, bm = kk < ncol ? b[m] : zero;
                    float2 z;
                    if (k == 0) {
                        z = make_float2(am.x, bm.x);
                    } else if (k == NC) {
                        z = make_float2(am.y, bm.y);
                    } else {
                        z = k < NC ? make_float2(am.x - bm.y, am.y + bm.x) : make_float2(am.x + bm.y, bm.x - am.y);
                    }
                    v[m] = z;
                }
            }
            FX::template dit<1>(v, ldr, trow, twx);
            float2 z[P];
#pragma unroll
            for (int m = 0; m < P; ++m) z[m] = cscale(v[m], p.inv_n);
            const DevChannel& C = p.ch[0];
            float2 w[P];
#pragma unroll
            for (int m = 0; m < P; ++m) w[m] = make_float2(0.f, 0.f);
            for (int k = 0; k < C.nprod; ++k) {
                const DevProd& pd = C.prod[k];
                const int pg = static_cast<int>(pd.pow[0]);
#pragma unroll
                for (int m = 0; m < P; ++m) {
                    float a = pd.coef, b = pd.coef;
                    for (int e = 0; e < pg; ++e) {
                        a *= z[m].x;
                        b *= z[m].y;
                    }
                    w[m].x += a;
                    w[m].y += b;
                }
            }
            FX::template dif<-1>(w, ldr, trow, twx);
            // unpack the pair's two rows into the packed columns
            float2* const W = ldr.wl;
            wave_lds_sync();
#pragma unroll
            for (int m = 0; m < P; ++m) W[drx + m * TX] = w[m];
            wave_lds_sync();
#pragma unroll
            for (int j = 0; j < NC / TX; ++j) {
                const int c = trow + j * TX;
#pragma unroll
                for (int rr = 0; rr < 2; ++rr) {
                    float2 o;
                    if (c == 0) {
                        const float2 a = W[0], b = W[NC];
                        o = rr ? make_float2(a.y, b.y) : make_float2(a.x, b.x);
                    } else {
                        const float2 a = W[c], b = W[LX - c];
                        o = rr ? make_float2(0.5f * (a.y + b.y), 0.5f * (b.x - a.x))
                               : make_float2(0.5f * (a.x + b.x), 0.5f * (a.y - b.y));
                    }
                    X[c * XS + p0 + rr] = o;
                }
            }
        }
        __syncthreads();
    }

    // state and channel array back to HBM; the counter moves on
#pragma unroll
    for (int r = 0; r < CR; ++r) {
        const int c = r * CPR + li;
        const size_t base = (static_cast<size_t>(c >> lt) * LY << lt) + (c & (tc - 1));
#pragma unroll
        for (int m = 0; m < P; ++m) gstore(Sg + base + static_cast<size_t>(tcol + m * TY) * tc, st[r][m]);
    }
    for (int i = tid; i < NC * LY; i += NTHR) {
        const int ct = i / (LY * tc), rem = i - ct * (LY * tc);
        const int y = rem >> lt, c = (ct << lt) + (rem & (tc - 1));
        gstore(Ng + i, X[c * XS + y]);
    }
    if (bad) atomicOr(mem.flag, bad);
    if (rl.advance && tid == 0) *mem.step_ctr += static_cast<uint64_t>(rl.nsteps);
}

// allow the resident kernels their LDS (above the default dynamic limit)
hipError_t resident_setup() {
#define PSS_RES_ATTR(AX, AY)                                                                                     \
    if (hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&resident_kernel<AX, AY>),              \
                                           hipFuncAttributeMaxDynamicSharedMemorySize,                            \
                                           static_cast<int>(resident_lds_bytes(AX, AY))))                        \
        return e;
    PSS_RES_ATTR(64, 64)
    PSS_RES_ATTR(64, 128)
    PSS_RES_ATTR(128, 64)
    PSS_RES_ATTR(128, 128)
#undef PSS_RES_ATTR
    return hipSuccess;
}

hipError_t launch_batch_resident(hipStream_t s, const ResidentLaunch& rl) {
    if (rl.nmem < 1 || rl.nsteps < 1) return hipSuccess;
    const size_t lds = resident_lds_bytes(rl.lx, rl.ly);
#define PSS_RES(AX, AY)                                                                                      if (rl.lx == AX && rl.ly == AY) {                                                                            hipLaunchKernelGGL((resident_kernel<AX, AY>), dim3(rl.nmem), dim3(resident_threads(AX, AY)), lds, s, rl);         return hipGetLastError();                                                                            }
    PSS_RES(64, 64)
    PSS_RES(64, 128)
    PSS_RES(128, 64)
    PSS_RES(128, 128)
#undef PSS_RES
    return hipErrorInvalidValue;
}

hipError_t launch_batch_update(hipStream_t s, const BatchLaunch& bl, size_t lds) {
    if (bl.ncls < 1 || bl.total < 1) return hipSuccess;
    hipLaunchKernelGGL(batch_update_kernel, dim3(bl.total), dim3(256), lds, s, bl);
    return hipGetLastError();
}

hipError_t launch_batch_xrow(hipStream_t s, const BatchLaunch& bl, size_t lds) {
    if (bl.ncls < 1 || bl.total < 1) return hipSuccess;
    hipLaunchKernelGGL(batch_xrow_kernel, dim3(bl.total), dim3(256), lds, s, bl);
    return hipGetLastError();
}
#endif  // PSS_BATCH

#if defined(PSS_COMMON)
#define PSS_DECL_L(L)                                                               \
    hipError_t launch_line1d_L##L(int mode, int nf, const LaunchArgs& a);          \
    hipError_t line1d_setup_L##L();                                                 \
    hipError_t launch_update_L##L(int mode, int nf, const LaunchArgs& a);          \
    hipError_t launch_ypass_L##L(int mode, const YArgs& ya, const LaunchArgs& a);  \
    hipError_t launch_xrow_L##L(int mode, int ng, const LaunchArgs& a);            \
    hipError_t launch_adjcol_L##L(int mode, const AdjArgs& aa, const LaunchArgs& a);
PSS_DECL_L(8)
PSS_DECL_L(16)
PSS_DECL_L(32)
PSS_DECL_L(64)
PSS_DECL_L(128)
PSS_DECL_L(256)
PSS_DECL_L(512)
PSS_DECL_L(1024)
PSS_DECL_L(2048)
PSS_DECL_L(4096)

int max_points(int L, int nregs) {
    const int cap = nregs <= 1 ? 16 : (nregs == 2 ? 8 : 4);
    return cap < L ? cap : L;
}

hipError_t launch_line1d(int mode, int N, int nf, const LaunchArgs& a) {
    switch (N) {
        case 8: return launch_line1d_L8(mode, nf, a);
        case 16: return launch_line1d_L16(mode, nf, a);
        case 32: return launch_line1d_L32(mode, nf, a);
        case 64: return launch_line1d_L64(mode, nf, a);
        case 128: return launch_line1d_L128(mode, nf, a);
        case 256: return launch_line1d_L256(mode, nf, a);
        case 512: return launch_line1d_L512(mode, nf, a);
        case 1024: return launch_line1d_L1024(mode, nf, a);
        case 2048: return launch_line1d_L2048(mode, nf, a);
        case 4096: return launch_line1d_L4096(mode, nf, a);
        default: return launch_line1d_mr(mode, N, nf, a.ng, a);
    }
}

hipError_t line1d_setup(int N) {
    switch (N) {
        case 8: return line1d_setup_L8();
        case 16: return line1d_setup_L16();
        case 32: return line1d_setup_L32();
        case 64: return line1d_setup_L64();
        case 128: return line1d_setup_L128();
        case 256: return line1d_setup_L256();
        case 512: return line1d_setup_L512();
        case 1024: return line1d_setup_L1024();
        case 2048: return line1d_setup_L2048();
        case 4096: return line1d_setup_L4096();
        default: return line1d_mr_setup();
    }
}

hipError_t launch_update(int mode, int L, int nf, const LaunchArgs& a) {
    switch (L) {
        case 8: return launch_update_L8(mode, nf, a);
        case 16: return launch_update_L16(mode, nf, a);
        case 32: return launch_update_L32(mode, nf, a);
        case 64: return launch_update_L64(mode, nf, a);
        case 128: return launch_update_L128(mode, nf, a);
        case 256: return launch_update_L256(mode, nf, a);
        case 512: return launch_update_L512(mode, nf, a);
        case 1024: return launch_update_L1024(mode, nf, a);
        case 2048: return launch_update_L2048(mode, nf, a);
        case 4096: return launch_update_L4096(mode, nf, a);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_ypass(int mode, int L, const YArgs& ya, const LaunchArgs& a) {
    switch (L) {
        case 8: return launch_ypass_L8(mode, ya, a);
        case 16: return launch_ypass_L16(mode, ya, a);
        case 32: return launch_ypass_L32(mode, ya, a);
        case 64: return launch_ypass_L64(mode, ya, a);
        case 128: return launch_ypass_L128(mode, ya, a);
        case 256: return launch_ypass_L256(mode, ya, a);
        case 512: return launch_ypass_L512(mode, ya, a);
        case 1024: return launch_ypass_L1024(mode, ya, a);
        case 2048: return launch_ypass_L2048(mode, ya, a);
        case 4096: return launch_ypass_L4096(mode, ya, a);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_xrow(int mode, int L, int ng, const LaunchArgs& a) {
    switch (L) {
        case 8: return launch_xrow_L8(mode, ng, a);
        case 16: return launch_xrow_L16(mode, ng, a);
        case 32: return launch_xrow_L32(mode, ng, a);
        case 64: return launch_xrow_L64(mode, ng, a);
        case 128: return launch_xrow_L128(mode, ng, a);
        case 256: return launch_xrow_L256(mode, ng, a);
        case 512: return launch_xrow_L512(mode, ng, a);
        case 1024: return launch_xrow_L1024(mode, ng, a);
        case 2048: return launch_xrow_L2048(mode, ng, a);
        case 4096: return launch_xrow_L4096(mode, ng, a);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_adjcol(int mode, int L, const AdjArgs& aa, const LaunchArgs& a) {
    switch (L) {
        case 8: return launch_adjcol_L8(mode, aa, a);
        case 16: return launch_adjcol_L16(mode, aa, a);
        case 32: return launch_adjcol_L32(mode, aa, a);
        case 64: return launch_adjcol_L64(mode, aa, a);
        case 128: return launch_adjcol_L128(mode, aa, a);
        case 256: return launch_adjcol_L256(mode, aa, a);
        case 512: return launch_adjcol_L512(mode, aa, a);
        case 1024: return launch_adjcol_L1024(mode, aa, a);
        case 2048: return launch_adjcol_L2048(mode, aa, a);
        case 4096: return launch_adjcol_L4096(mode, aa, a);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_adjseed(hipStream_t s, const float2* phi, float2* g, const float* coef, int nshell, int nx, int ny,
                          int tc) {
    const int64_t total = static_cast<int64_t>(nx / 2) * ny;
    hipLaunchKernelGGL(adjseed_kernel, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0, s, phi, g, coef,
                       nshell, nx, ny, tc);
    return hipGetLastError();
}

hipError_t launch_advance(hipStream_t s, uint64_t* step_ctr, int64_t k) {
    hipLaunchKernelGGL(advance_kernel, dim3(1), dim3(64), 0, s, step_ctr, k);
    return hipGetLastError();
}

hipError_t launch_advance_many(hipStream_t s, uint64_t* const* ctrs, int n, int64_t k) {
    if (n < 1) return hipSuccess;
    hipLaunchKernelGGL(advance_many_kernel, dim3((n + 255) / 256), dim3(256), 0, s, ctrs, n, k);
    return hipGetLastError();
}

hipError_t launch_apply_frame(hipStream_t s, float* real, const int2* frame, int n) {
    if (n < 1) return hipSuccess;
    hipLaunchKernelGGL(apply_frame_kernel, dim3((n + 255) / 256), dim3(256), 0, s, real, frame, n);
    return hipGetLastError();
}

hipError_t launch_take_flags(hipStream_t s, uint64_t* const* ctrs, int n, uint32_t* out) {
    if (n < 1) return hipSuccess;
    hipLaunchKernelGGL(take_flags_kernel, dim3((n + 255) / 256), dim3(256), 0, s, ctrs, n, out);
    return hipGetLastError();
}

hipError_t launch_init_uniform(hipStream_t s, float* out, int64_t n, uint32_t field, uint32_t key0, uint32_t key1,
                               double lo, double hi) {
    const int64_t blocks = (n + 255) / 256;
    hipLaunchKernelGGL(init_uniform_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, out, n, field, key0,
                       key1, lo, hi);
    return hipGetLastError();
}

hipError_t launch_shells(hipStream_t s, const float2* S, int nx, int ny, int nz, int tc, int ndim, double scale,
                         int nshell, unsigned long long* acc) {
    if (nshell < 1) return hipSuccess;
    unsigned long long* hi = acc;
    unsigned long long* lo = acc + nshell;
    unsigned long long* cnt = acc + 2 * nshell;
    auto* key = reinterpret_cast<unsigned int*>(acc + 3 * nshell);
    hipLaunchKernelGGL(shell_keys_kernel, dim3(256), dim3(256), sizeof(unsigned int) * nshell, s, S, nx, ny, nz, tc,
                       ndim, scale, nshell, key);
    const size_t lds = nshell * (2 * sizeof(unsigned long long) + 2 * sizeof(unsigned int));
    hipLaunchKernelGGL(shell_sums_kernel, dim3(256), dim3(256), lds, s, S, nx, ny, nz, tc, ndim, scale, nshell, key,
                       hi, lo, cnt);
    hipLaunchKernelGGL(shell_means_kernel, dim3((nshell + 255) / 256), dim3(256), 0, s, nshell, key, hi, lo, cnt);
    return hipGetLastError();
}

hipError_t launch_philox(hipStream_t s, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                         int64_t count, uint32_t* out) {
    const int64_t blocks = (count + 255) / 256;
    hipLaunchKernelGGL(philox_kernel, dim3(static_cast<unsigned>(blocks)), dim3(256), 0, s, c0, c1, c2, c3, k0, k1,
                       count, out);
    return hipGetLastError();
}

#endif  // PSS_COMMON

}  // namespace pss
