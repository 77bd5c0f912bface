// HIP kernels of the pseudo-spectral stochastic step for gfx950.
//
// One 2D step (eq:timeupdate and the six-step list after it) is two kernels:
//
//   update kernel (lines along y, one tile of TC packed columns per block)
//     forward y-FFT of every product channel  -> N_hat(kx, ky)       (step 4)
//     Philox4x32-10 + Box-Muller noise per mode, in registers        (step 5)
//     phi <- (phi + dt sum M N_hat + sigma xi) / (1 - dt L)          (step 6)
//     de-alias mask, inverse y-FFT of every factor field  -> V       (steps 2-3)
//   x kernel (lines along x, RB rows per block, two real rows per complex FFT)
//     inverse x-FFT of V (C2R) -> u(x, y); products sum c prod u^p   (step 3)
//     forward x-FFT (R2C) -> channel arrays for the next step        (step 4)
//
// The spectral arrays use the packed half-spectrum layout described in
// pss_plan.h: column 0 holds X(kx=0) + i X(kx=Nx/2).
#include <hip/hip_runtime.h>

#include "pss_device.h"
#include "pss_kernels.h"
#include "pss_plan.h"

namespace pss {

// ----------------------------------------------------------------- modes
struct ModeQ {
    float q2, invq;
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
    m.invq = m.q2 > 0.f ? 1.f / sqrtf(m.q2) : 0.f;
    m.iq[0] = (kx == -(p.n[0] >> 1)) ? 0.f : qx;
    m.iq[1] = (ky == -(p.n[1] >> 1)) ? 0.f : qy;
    m.iq[2] = (p.n[2] > 1 && kz == -(p.n[2] >> 1)) ? 0.f : qz;
    return m;
}

// sum_m coef (q^2)^a |q|^-b (i qx)^cx (i qy)^cy (i qz)^cz
__device__ __forceinline__ float2 eval_op(const DevOp& op, const ModeQ& q) {
    float re = 0.f, im = 0.f;
    for (int i = 0; i < op.n; ++i) {
        const DevMono mo = op.m[i];
        float s = mo.coef;
        for (int e = 0; e < mo.q2; ++e) s *= q.q2;
        for (int e = 0; e < mo.invq; ++e) s *= q.invq;
        for (int e = 0; e < mo.ix; ++e) s *= q.iq[0];
        for (int e = 0; e < mo.iy; ++e) s *= q.iq[1];
        for (int e = 0; e < mo.iz; ++e) s *= q.iq[2];
        switch (mo.ipow) {
            case 0: re += s; break;
            case 1: im += s; break;
            case 2: re -= s; break;
            default: im -= s; break;
        }
    }
    return make_float2(re, im);
}

// 1 / (1 - dt L(q))
__device__ __forceinline__ float2 implicit_inv(const DevPlan& p, int f, const ModeQ& q) {
    const float2 L = eval_op(p.implicit_op[f], q);
    const float ar = 1.f - p.dt * L.x, ai = -p.dt * L.y;
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

// Scaled unit white noise sigma(q) xi_hat(k) of field f at step `step` for a
// mode with full-spectrum linear index lin and negative-mode index lneg.
__device__ __forceinline__ float2 noise_mode(const DevPlan& p, int f, uint32_t step, uint32_t lin,
                                             uint32_t lneg, const ModeQ& q) {
    const float D = eval_op(p.noise_op[f], q).x;
    const uint32_t c = lin < lneg ? lin : lneg;
    const uint4 w = philox4x32_10(make_uint4(c, step, static_cast<uint32_t>(f), 0u), p.key0, p.key1);
    const float2 g = box_muller(w.x, w.y);
    const float sd = sqrtf(fmaxf(D, 0.f));
    if (lin == lneg) return make_float2(p.amp_self * sd * g.x, 0.f);
    const float a = p.amp_pair * sd;
    return lin == c ? make_float2(a * g.x, a * g.y) : make_float2(a * g.x, -a * g.y);
}

// full-spectrum linear index of mode (kx, ky, kz), each in [0, n_i)
__device__ __forceinline__ uint32_t lin_index(const DevPlan& p, int kx, int ky, int kz) {
    return (static_cast<uint32_t>(kz) * p.n[1] + ky) * p.n[0] + kx;
}
__device__ __forceinline__ uint32_t lin_neg(const DevPlan& p, int kx, int ky, int kz) {
    const int nx = p.n[0], ny = p.n[1], nz = p.n[2];
    return lin_index(p, (nx - kx) & (nx - 1), (ny - ky) & (ny - 1), (nz - kz) & (nz - 1));
}

// select element F of a register array with a runtime index (unrolled)
template <int NF, int P>
__device__ __forceinline__ float2 pick(const float2 (&a)[NF][P], int f, int m) {
    float2 r = a[0][m];
#pragma unroll
    for (int i = 1; i < NF; ++i)
        if (f == i) r = a[i][m];
    return r;
}

template <int NF, int P>
__device__ __forceinline__ void add_to(float2 (&a)[NF][P], int f, int m, float2 v) {
#pragma unroll
    for (int i = 0; i < NF; ++i)
        if (f == i) a[i][m] = cadd(a[i][m], v);
}

// ------------------------------------------------------------ update kernel
// Lines along the last axis u (y in 2D).  Block = one tile of TC packed
// columns; thread (cc, t) holds u = t + m*T of column ct*TC + cc in v[m].
// Array element (column c, u) of the tile is at  tile_base + u*TC + cc  with
// tile_base = ct * (L*TC).
//
// Column 0 holds S = phi(0,k) + i phi(Nx/2,k) with both parts Hermitian along
// u; its threads unpack with the partner value at -u, which they exchange
// through LDS (tile 0 only, block-uniform barriers).  LDS layout:
//   TC line buffers | acc0[NF*L] | accn[NF*L] | old[NF*L] (= channel exchange)
template <int L, int P, int NF, int MODE>
__global__ void __launch_bounds__(256) update_kernel(const DevPlan* __restrict__ plan, Bufs bufs, Geo geo,
                                                      const uint64_t* __restrict__ step_ctr,
                                                      int step_off, const float2* __restrict__ tw) {
    constexpr int T = L / P;
    extern __shared__ float2 smem[];
    const DevPlan& p = *plan;
    const int tc = geo.tc;
    const int tid = threadIdx.x;
    const int cc = tid % tc;
    const int t = tid / tc;
    const int ct = blockIdx.x;    // tile index
    const int c = ct * tc + cc;   // packed column
    const size_t base = static_cast<size_t>(ct) * (L * tc) + cc;
    float2* line = smem + cc * lds_line(L);
    float2* acc0 = smem + tc * lds_line(L);  // kx = 0 accumulators, then new phi(0,k)
    float2* accn = acc0 + NF * L;            // kx = Nx/2 accumulators, then new phi(Nx/2,k)
    float2* oldb = accn + NF * L;            // old column-0 state
    float2* xbuf = oldb;                     // channel exchange; done before oldb is written
    const bool col0 = (c == 0);
    const bool tile0 = (ct == 0);
    const int nx = p.n[0];
    const int nf = p.nf;

    if constexpr (MODE == MODE_FWD_STORE) {
        // forward transform of an x-transformed array, stored as the state
        float2 v[P];
#pragma unroll
        for (int m = 0; m < P; ++m) v[m] = bufs.in[base + (t + m * T) * tc];
        fft_line<L, P, -1>(v, line, t, tw);
#pragma unroll
        for (int m = 0; m < P; ++m) bufs.S[bufs.sel][base + (t + m * T) * tc] = v[m];
        return;
    }
    if constexpr (MODE == MODE_INV_OUT) {
        float2 v[P];
#pragma unroll
        for (int m = 0; m < P; ++m) v[m] = bufs.S[bufs.sel][base + (t + m * T) * tc];
        fft_line<L, P, 1>(v, line, t, tw);
#pragma unroll
        for (int m = 0; m < P; ++m) bufs.out[base + (t + m * T) * tc] = v[m];
        return;
    }

    // ---- MODE_STEP or MODE_PROLOGUE
    // Column-0 threads keep everything in LDS and loop over their modes at run
    // time; the other threads keep register arrays indexed by constants.
    const uint32_t step = static_cast<uint32_t>(*step_ctr) + static_cast<uint32_t>(step_off);
    float2 s[NF][P];    // state, then new state
    float2 acc[NF][P];  // explicit contributions at kx = c
#pragma unroll
    for (int f = 0; f < NF; ++f)
#pragma unroll
        for (int m = 0; m < P; ++m) acc[f][m] = make_float2(0.f, 0.f);

    if constexpr (MODE == MODE_STEP) {
        if (col0)
            for (int i = t; i < NF * L; i += T) {
                acc0[i] = make_float2(0.f, 0.f);
                accn[i] = make_float2(0.f, 0.f);
            }
        // explicit real-space channels
        for (int ch = 0; ch < p.nch; ++ch) {
            const DevChannel& C = p.ch[ch];
            float2 v[P];
#pragma unroll
            for (int m = 0; m < P; ++m) v[m] = bufs.N[ch][base + (t + m * T) * tc];
            fft_line<L, P, -1>(v, line, t, tw);
            if (tile0) {
                if (col0) {
#pragma unroll
                    for (int m = 0; m < P; ++m) xbuf[t + m * T] = v[m];
                }
                __syncthreads();
                if (col0) {
#pragma unroll 1
                    for (int m = 0; m < P; ++m) {
                        const int u = t + m * T;
                        const float2 a = xbuf[u], b = xbuf[(L - u) & (L - 1)];
                        // unpack the kx = 0 and kx = Nx/2 parts
                        const float2 n0 = make_float2(0.5f * (a.x + b.x), 0.5f * (a.y - b.y));
                        const float2 nn = make_float2(0.5f * (a.y + b.y), 0.5f * (b.x - a.x));
                        const int ku = signed_mode(u, L);
                        const int o = C.target * L + u;
                        acc0[o] = cadd(acc0[o], cmul(eval_op(C.op, mode_q(p, 0, ku, 0)), n0));
                        accn[o] = cadd(accn[o], cmul(eval_op(C.op, mode_q(p, -(nx >> 1), ku, 0)), nn));
                    }
                }
                __syncthreads();
            }
            if (!col0) {
#pragma unroll
                for (int m = 0; m < P; ++m) {
                    const ModeQ q = mode_q(p, c, signed_mode(t + m * T, L), 0);
                    add_to(acc, C.target, m, cmul(eval_op(C.op, q), v[m]));
                }
            }
        }
    }

    // old state; column 0 parks it in LDS for the partner reads
#pragma unroll
    for (int f = 0; f < NF; ++f) {
        if (f < nf) {
#pragma unroll
            for (int m = 0; m < P; ++m) s[f][m] = bufs.S[f][base + (t + m * T) * tc];
        } else {
#pragma unroll
            for (int m = 0; m < P; ++m) s[f][m] = make_float2(0.f, 0.f);
        }
        if (col0) {
#pragma unroll
            for (int m = 0; m < P; ++m) oldb[f * L + t + m * T] = s[f][m];
        }
    }
    if (tile0) __syncthreads();

    if (!col0) {
        if constexpr (MODE == MODE_STEP) {
            // Fourier-space terms with a single linear factor
            for (int d = 0; d < p.nd; ++d) {
                const DevDirect& Dd = p.direct[d];
#pragma unroll
                for (int m = 0; m < P; ++m) {
                    const ModeQ q = mode_q(p, c, signed_mode(t + m * T, L), 0);
                    add_to(acc, Dd.target, m, cmul(eval_op(Dd.op, q), pick(s, Dd.src, m)));
                }
            }
            // semi-implicit update with noise
#pragma unroll
            for (int f = 0; f < NF; ++f) {
                if (f >= nf) continue;
                const bool noisy = p.noisy[f] != 0;
#pragma unroll
                for (int m = 0; m < P; ++m) {
                    const int u = t + m * T;
                    const ModeQ q = mode_q(p, c, signed_mode(u, L), 0);
                    float2 r = cadd(s[f][m], cscale(acc[f][m], p.dt));
                    if (noisy) r = cadd(r, noise_mode(p, f, step, lin_index(p, c, u, 0), lin_neg(p, c, u, 0), q));
                    s[f][m] = cmul(r, implicit_inv(p, f, q));
                    bufs.S[f][base + u * tc] = s[f][m];
                }
            }
        }
    } else {
        // column 0: unpack S = phi(0,k) + i phi(Nx/2,k) with the partner -u
        if constexpr (MODE == MODE_STEP) {
            for (int d = 0; d < p.nd; ++d) {
                const DevDirect& Dd = p.direct[d];
#pragma unroll 1
                for (int m = 0; m < P; ++m) {
                    const int u = t + m * T;
                    const int ku = signed_mode(u, L);
                    const float2 a = oldb[Dd.src * L + u], b = oldb[Dd.src * L + ((L - u) & (L - 1))];
                    const float2 n0 = make_float2(0.5f * (a.x + b.x), 0.5f * (a.y - b.y));
                    const float2 nn = make_float2(0.5f * (a.y + b.y), 0.5f * (b.x - a.x));
                    const int o = Dd.target * L + u;
                    acc0[o] = cadd(acc0[o], cmul(eval_op(Dd.op, mode_q(p, 0, ku, 0)), n0));
                    accn[o] = cadd(accn[o], cmul(eval_op(Dd.op, mode_q(p, -(nx >> 1), ku, 0)), nn));
                }
            }
        }
        for (int f = 0; f < nf; ++f) {
            const bool noisy = p.noisy[f] != 0;
#pragma unroll 1
            for (int m = 0; m < P; ++m) {
                const int u = t + m * T;
                const int ku = signed_mode(u, L);
                const float2 a = oldb[f * L + u], b = oldb[f * L + ((L - u) & (L - 1))];
                float2 s0 = make_float2(0.5f * (a.x + b.x), 0.5f * (a.y - b.y));
                float2 sn = make_float2(0.5f * (a.y + b.y), 0.5f * (b.x - a.x));
                if constexpr (MODE == MODE_STEP) {
                    const ModeQ q0 = mode_q(p, 0, ku, 0);
                    const ModeQ qn = mode_q(p, -(nx >> 1), ku, 0);
                    s0 = cadd(s0, cscale(acc0[f * L + u], p.dt));
                    sn = cadd(sn, cscale(accn[f * L + u], p.dt));
                    if (noisy) {
                        s0 = cadd(s0, noise_mode(p, f, step, lin_index(p, 0, u, 0), lin_neg(p, 0, u, 0), q0));
                        sn = cadd(sn, noise_mode(p, f, step, lin_index(p, nx >> 1, u, 0),
                                                 lin_neg(p, nx >> 1, u, 0), qn));
                    }
                    s0 = cmul(s0, implicit_inv(p, f, q0));
                    sn = cmul(sn, implicit_inv(p, f, qn));
                    bufs.S[f][base + u * tc] = make_float2(s0.x - sn.y, s0.y + sn.x);  // s0 + i sn
                }
                // own slots only: the new halves for the inverse transforms
                acc0[f * L + u] = s0;
                accn[f * L + u] = sn;
            }
        }
    }

    // de-aliased inverse transforms of every factor field
    for (int g = 0; g < p.ng; ++g) {
        const DevMask& mk = p.mask[g];
        if (ct * tc >= mk.ncol) continue;  // whole tile masked: never read
        const int fg = p.gfield[g];
        float2 v[P];
        if (!col0) {
#pragma unroll
            for (int m = 0; m < P; ++m)
                v[m] = mask_keep(mk, c, signed_mode(t + m * T, L), 0) ? pick(s, fg, m) : make_float2(0.f, 0.f);
        } else {
#pragma unroll
            for (int m = 0; m < P; ++m) {
                const int u = t + m * T;
                const int ku = signed_mode(u, L);
                const float2 z0 = mask_keep(mk, 0, ku, 0) ? acc0[fg * L + u] : make_float2(0.f, 0.f);
                const float2 zn = mask_keep(mk, -(nx >> 1), ku, 0) ? accn[fg * L + u] : make_float2(0.f, 0.f);
                v[m] = make_float2(z0.x - zn.y, z0.y + zn.x);
            }
        }
        fft_line<L, P, 1>(v, line, t, tw);
#pragma unroll
        for (int m = 0; m < P; ++m) bufs.V[g][base + (t + m * T) * tc] = v[m];
    }
}

// ----------------------------------------------------------------- x kernel
// Rows of length L = Nx; block = RB consecutive rows, pair p = rows (2p, 2p+1)
// packed as one complex line.  Packed-column arrays are read and written in
// whole tile blocks of RB*TC contiguous elements.
template <int L, int P, int NG, int MODE>
__global__ void __launch_bounds__(256) xrow_kernel(const DevPlan* __restrict__ plan, Bufs bufs, Geo geo,
                                                    const float2* __restrict__ tw) {
    constexpr int T = L / P;
    constexpr int NC = L / 2;  // packed columns
    extern __shared__ float2 smem[];
    const DevPlan& p = *plan;
    const int tc = geo.tc, rb = geo.rb;
    const int ntile = NC / tc;
    const int tid = threadIdx.x;
    const int nthr = blockDim.x;
    const int pr = tid / T;  // pair within the block
    const int t = tid % T;
    const int y0 = blockIdx.x * rb;  // first row (2D: y)
    const int ny = p.n[1];
    float2* line = smem + pr * lds_line(L);
    float2* stage = smem + (rb / 2) * lds_line(L);  // rb x NC (+pad)
    const int spitch = NC + 1;

    // load packed columns [0, ncol) of rows y0..y0+rb-1 into stage
    auto stage_rows = [&](const float2* __restrict__ src, int ncol) {
        const int nt = (ncol + tc - 1) / tc;
        const int per = rb * tc;
        for (int i = tid; i < nt * per; i += nthr) {
            const int tl = i / per, rem = i - tl * per;
            const int r = rem / tc, cc = rem - r * tc;
            stage[r * spitch + tl * tc + cc] = src[(static_cast<size_t>(tl) * ny + y0 + r) * tc + cc];
        }
    };
    // build the packed complex input Z[k] = X_row0[k] + i X_row1[k] of pair pr
    auto build_z = [&](float2 (&v)[P], int ncol) {
        const float2* r0 = stage + (2 * pr) * spitch;
        const float2* r1 = r0 + spitch;
#pragma unroll
        for (int m = 0; m < P; ++m) {
            const int k = t + m * T;
            float2 z;
            if (k == 0) {
                z = make_float2(r0[0].x, r1[0].x);
            } else if (k == NC) {
                z = make_float2(r0[0].y, r1[0].y);
            } else {
                const int kk = k < NC ? k : L - k;
                const float2 a = kk < ncol ? r0[kk] : make_float2(0.f, 0.f);
                const float2 b = kk < ncol ? r1[kk] : make_float2(0.f, 0.f);
                z = k < NC ? make_float2(a.x - b.y, a.y + b.x) : make_float2(a.x + b.y, b.x - a.y);
            }
            v[m] = z;
        }
    };
    // unpack the forward transform W of each pair and store packed columns
    auto store_rows = [&](float2* __restrict__ dst) {
        const int per = rb * tc;
        for (int i = tid; i < ntile * per; i += nthr) {
            const int tl = i / per, rem = i - tl * per;
            const int r = rem / tc, cc = rem - r * tc;
            const int c = tl * tc + cc;
            const float2* W = smem + (r >> 1) * lds_line(L);
            float2 o;
            if (c == 0) {
                const float2 a = W[lds_pad(0)], b = W[lds_pad(NC)];
                o = (r & 1) ? make_float2(a.y, b.y) : make_float2(a.x, b.x);
            } else {
                const float2 a = W[lds_pad(c)], b = W[lds_pad(L - c)];
                o = (r & 1) ? make_float2(0.5f * (a.y + b.y), 0.5f * (b.x - a.x))
                            : make_float2(0.5f * (a.x + b.x), 0.5f * (a.y - b.y));
            }
            dst[(static_cast<size_t>(tl) * ny + y0 + r) * tc + cc] = o;
        }
    };

    if constexpr (MODE == MODE_R2C_IN) {
        // real rows -> packed columns (forward transform, unnormalised)
        const float* __restrict__ src = bufs.real_in;
        float2 v[P];
#pragma unroll
        for (int m = 0; m < P; ++m) {
            const int x = t + m * T;
            v[m] = make_float2(src[static_cast<size_t>(y0 + 2 * pr) * L + x],
                               src[static_cast<size_t>(y0 + 2 * pr + 1) * L + x]);
        }
        fft_line<L, P, -1>(v, line, t, tw);
#pragma unroll
        for (int m = 0; m < P; ++m) line[lds_pad(t + m * T)] = v[m];
        __syncthreads();
        store_rows(bufs.out);
        return;
    }
    if constexpr (MODE == MODE_C2R_OUT) {
        stage_rows(bufs.in, NC);
        __syncthreads();
        float2 v[P];
        build_z(v, NC);
        fft_line<L, P, 1>(v, line, t, tw);
        float* __restrict__ dst = bufs.real_out;
#pragma unroll
        for (int m = 0; m < P; ++m) {
            const int x = t + m * T;
            dst[static_cast<size_t>(y0 + 2 * pr) * L + x] = v[m].x * p.inv_n;
            dst[static_cast<size_t>(y0 + 2 * pr + 1) * L + x] = v[m].y * p.inv_n;
        }
        return;
    }

    // MODE_STEP: real-space values of every factor field
    float2 z[NG][P];
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        const int ncol = p.mask[g].ncol;
        stage_rows(bufs.V[g], ncol);
        __syncthreads();
        float2 v[P];
        build_z(v, ncol);
        __syncthreads();  // stage is reused by the next factor
        fft_line<L, P, 1>(v, line, t, tw);
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
            const DevProd pd = C.prod[k];
#pragma unroll
            for (int m = 0; m < P; ++m) {
                float a = pd.coef, b = pd.coef;
#pragma unroll
                for (int g = 0; g < NG; ++g)
                    for (int e = 0; e < pd.pow[g]; ++e) {
                        a *= z[g][m].x;
                        b *= z[g][m].y;
                    }
                w[m].x += a;
                w[m].y += b;
            }
        }
        fft_line<L, P, -1>(w, line, t, tw);
#pragma unroll
        for (int m = 0; m < P; ++m) line[lds_pad(t + m * T)] = w[m];
        __syncthreads();
        store_rows(bufs.N[ch]);
        __syncthreads();
    }
}

#if defined(PSS_COMMON)
// ---------------------------------------------------------------- utilities
__global__ void advance_kernel(uint64_t* step_ctr, int64_t k) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *step_ctr += static_cast<uint64_t>(k);
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
// kx = Nx/2 (weight 1 each) with the partner element at -y.
__device__ __forceinline__ void shell_add(double* sums, unsigned int* cnt, int nshell, int kx, int ky, int kz,
                                          double v, unsigned int w) {
    const double kk = static_cast<double>(kx) * kx + static_cast<double>(ky) * ky + static_cast<double>(kz) * kz;
    const int j = static_cast<int>(rint(sqrt(kk)));
    if (j >= 1 && j < nshell) {
        atomicAdd(&sums[j], v * w);
        atomicAdd(&cnt[j], w);
    }
}

__global__ void shells_kernel(const float2* __restrict__ S, int nx, int ny, int tc, double scale, int nshell,
                              double* __restrict__ gsum, unsigned long long* __restrict__ gcnt) {
    extern __shared__ double lsum[];
    unsigned int* lcnt = reinterpret_cast<unsigned int*>(lsum + nshell);
    for (int i = threadIdx.x; i < nshell; i += blockDim.x) {
        lsum[i] = 0.0;
        lcnt[i] = 0u;
    }
    __syncthreads();
    const int ncols = nx / 2;
    const int64_t total = static_cast<int64_t>(ncols) * ny;
    for (int64_t e = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; e < total;
         e += static_cast<int64_t>(gridDim.x) * blockDim.x) {
        const int cc = static_cast<int>(e % tc);
        const int64_t r = e / tc;
        const int y = static_cast<int>(r % ny);
        const int ct = static_cast<int>(r / ny);
        const int c = ct * tc + cc;
        const int ky = y < ny / 2 ? y : y - ny;
        const float2 a = S[e];
        if (c > 0) {
            const double v = scale * (static_cast<double>(a.x) * a.x + static_cast<double>(a.y) * a.y);
            shell_add(lsum, lcnt, nshell, c, ky, 0, v, 2u);
        } else {
            const float2 b = S[static_cast<int64_t>((ny - y) & (ny - 1)) * tc];
            const double r0 = 0.5 * (static_cast<double>(a.x) + b.x), i0 = 0.5 * (static_cast<double>(a.y) - b.y);
            const double rn = 0.5 * (static_cast<double>(a.y) + b.y), in = 0.5 * (static_cast<double>(b.x) - a.x);
            shell_add(lsum, lcnt, nshell, 0, ky, 0, scale * (r0 * r0 + i0 * i0), 1u);
            shell_add(lsum, lcnt, nshell, -(nx / 2), ky, 0, scale * (rn * rn + in * in), 1u);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nshell; i += blockDim.x) {
        if (lcnt[i]) {
            atomicAdd(&gsum[i], lsum[i]);
            atomicAdd(&gcnt[i], static_cast<unsigned long long>(lcnt[i]));
        }
    }
}
#endif  // PSS_COMMON

// ------------------------------------------------------- launch dispatch
// This file is compiled once per line length with -DPSS_LINE_LEN=<L> (the
// kernels of that length) and once with -DPSS_COMMON (utilities and the
// length dispatch), so the instantiations build in parallel.
#if defined(PSS_LINE_LEN)
template <int L, int P, int NF>
static hipError_t launch_update_t(int mode, const LaunchArgs& a) {
    const int threads = a.geo.tc * (L / P);
    const size_t lds = update_lds_bytes(L, NF, a.geo.tc);
    dim3 grid(a.geo.ntile), block(threads);
    switch (mode) {
        case MODE_STEP:
            hipLaunchKernelGGL((update_kernel<L, P, NF, MODE_STEP>), grid, block, lds, a.stream, a.plan, a.bufs,
                               a.geo, a.step_ctr, a.step_off, a.tw_u);
            break;
        case MODE_PROLOGUE:
            hipLaunchKernelGGL((update_kernel<L, P, NF, MODE_PROLOGUE>), grid, block, lds, a.stream, a.plan,
                               a.bufs, a.geo, a.step_ctr, a.step_off, a.tw_u);
            break;
        case MODE_FWD_STORE:
            hipLaunchKernelGGL((update_kernel<L, P, 1, MODE_FWD_STORE>), grid, block, lds, a.stream, a.plan,
                               a.bufs, a.geo, a.step_ctr, a.step_off, a.tw_u);
            break;
        case MODE_INV_OUT:
            hipLaunchKernelGGL((update_kernel<L, P, 1, MODE_INV_OUT>), grid, block, lds, a.stream, a.plan,
                               a.bufs, a.geo, a.step_ctr, a.step_off, a.tw_u);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int L, int P, int NG>
static hipError_t launch_xrow_t(int mode, const LaunchArgs& a) {
    const int threads = (a.geo.rb / 2) * (L / P);
    const size_t lds = xrow_lds_bytes(L, a.geo.rb);
    dim3 grid(a.geo.nrowblk), block(threads);
    switch (mode) {
        case MODE_STEP:
            hipLaunchKernelGGL((xrow_kernel<L, P, NG, MODE_STEP>), grid, block, lds, a.stream, a.plan, a.bufs,
                               a.geo, a.tw_x);
            break;
        case MODE_R2C_IN:
            hipLaunchKernelGGL((xrow_kernel<L, P, 1, MODE_R2C_IN>), grid, block, lds, a.stream, a.plan, a.bufs,
                               a.geo, a.tw_x);
            break;
        case MODE_C2R_OUT:
            hipLaunchKernelGGL((xrow_kernel<L, P, 1, MODE_C2R_OUT>), grid, block, lds, a.stream, a.plan, a.bufs,
                               a.geo, a.tw_x);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

#define PSS_CAT2(a, b) a##b
#define PSS_CAT(a, b) PSS_CAT2(a, b)

hipError_t PSS_CAT(launch_update_L, PSS_LINE_LEN)(int mode, int nf, const LaunchArgs& a) {
    constexpr int L = PSS_LINE_LEN;
    constexpr int P = points_per_thread(L, 1);
    if (mode == MODE_FWD_STORE || mode == MODE_INV_OUT) return launch_update_t<L, P, 1>(mode, a);
    switch (nf) {
        case 1: return launch_update_t<L, P, 1>(mode, a);
        case 2: return launch_update_t<L, points_per_thread(L, 2), 2>(mode, a);
        case 3:
        case 4: return launch_update_t<L, points_per_thread(L, 4), 4>(mode, a);
        default: return hipErrorInvalidValue;
    }
}

hipError_t PSS_CAT(launch_xrow_L, PSS_LINE_LEN)(int mode, int ng, const LaunchArgs& a) {
    constexpr int L = PSS_LINE_LEN;
    constexpr int P = points_per_thread(L, 1);
    if (mode != MODE_STEP) return launch_xrow_t<L, P, 1>(mode, a);
    switch (ng) {
        case 0:
        case 1: return launch_xrow_t<L, P, 1>(mode, a);
        case 2: return launch_xrow_t<L, points_per_thread(L, 2), 2>(mode, a);
        case 3: return launch_xrow_t<L, points_per_thread(L, 4), 3>(mode, a);
        case 4: return launch_xrow_t<L, points_per_thread(L, 4), 4>(mode, a);
        default: return hipErrorInvalidValue;
    }
}
#endif  // PSS_LINE_LEN

#if defined(PSS_COMMON)
#define PSS_DECL_L(L)                                                         \
    hipError_t launch_update_L##L(int mode, int nf, const LaunchArgs& a);    \
    hipError_t launch_xrow_L##L(int mode, int ng, const LaunchArgs& a);
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

int update_threads(int L, int nf, int tc) {
    const int k = nf <= 1 ? 1 : (nf == 2 ? 2 : 4);
    return tc * (L / points_per_thread(L, k));
}

int xrow_threads(int L, int ng, int rb) {
    const int k = ng <= 1 ? 1 : (ng == 2 ? 2 : 4);
    return (rb / 2) * (L / points_per_thread(L, k));
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

hipError_t launch_advance(hipStream_t s, uint64_t* step_ctr, int64_t k) {
    hipLaunchKernelGGL(advance_kernel, dim3(1), dim3(64), 0, s, step_ctr, k);
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
                         int nshell, double* sums, unsigned long long* counts) {
    if (ndim != 2 || nz != 1) return hipErrorInvalidValue;
    const size_t lds = nshell * (sizeof(double) + sizeof(unsigned int));
    hipLaunchKernelGGL(shells_kernel, dim3(256), dim3(256), lds, s, S, nx, ny, tc, scale, nshell, sums, counts);
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
