// Device building blocks for the pseudo-spectral step on gfx950:
//   * complex helpers and in-register DFTs of size 2, 4, 8, 16 (the line
//     transforms built from them are in pss_fft.h);
//   * global-memory access helpers and the XCD-aware block order;
//   * Philox4x32-10 (Salmon et al., SC'11) and Box-Muller (1958).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pss {

// ------------------------------------------------------------------ complex
__device__ __forceinline__ float2 cadd(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ float2 cmul(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cscale(float2 a, float s) { return make_float2(a.x * s, a.y * s); }
__device__ __forceinline__ float2 cconj(float2 a) { return make_float2(a.x, -a.y); }

// multiply by DIR * i (DIR = -1: forward transform sign, +1: inverse)
template <int DIR>
__device__ __forceinline__ float2 mul_dir_i(float2 a) {
    return DIR > 0 ? make_float2(-a.y, a.x) : make_float2(a.y, -a.x);
}

// cos and sin of 2 pi j / 16 for j = 0..15 (multiples of pi/8)
#define PSS_C16 0.92387953251128675613f
#define PSS_S16 0.38268343236508977173f
#define PSS_C8 0.70710678118654752440f

template <int J>
struct Unit16 {
    static constexpr int j = J & 15;
    static constexpr float c = (j == 0) ? 1.f : (j == 1) ? PSS_C16 : (j == 2) ? PSS_C8 : (j == 3) ? PSS_S16
                             : (j == 4) ? 0.f : (j == 5) ? -PSS_S16 : (j == 6) ? -PSS_C8 : (j == 7) ? -PSS_C16
                             : (j == 8) ? -1.f : (j == 9) ? -PSS_C16 : (j == 10) ? -PSS_C8 : (j == 11) ? -PSS_S16
                             : (j == 12) ? 0.f : (j == 13) ? PSS_S16 : (j == 14) ? PSS_C8 : PSS_C16;
};

// a * exp(DIR * 2 pi i J / 16)
template <int DIR, int J>
__device__ __forceinline__ float2 rot16(float2 a) {
    constexpr int j = J & 15;
    if constexpr (j == 0) {
        return a;
    } else if constexpr (j == 4) {
        return mul_dir_i<DIR>(a);
    } else if constexpr (j == 8) {
        return make_float2(-a.x, -a.y);
    } else if constexpr (j == 12) {
        return mul_dir_i<-DIR>(a);
    } else {
        constexpr float c = Unit16<j>::c;
        constexpr float s = (DIR > 0 ? 1.f : -1.f) * Unit16<(j + 12) & 15>::c;
        return make_float2(a.x * c - a.y * s, a.x * s + a.y * c);
    }
}

// In-register DFT of size R: a[k] <- sum_r a[r] exp(DIR 2 pi i r k / R), natural order.
template <int R, int DIR>
struct DFT;

template <int DIR>
struct DFT<1, DIR> {
    static __device__ __forceinline__ void run(float2*) {}
};

template <int DIR>
struct DFT<2, DIR> {
    static __device__ __forceinline__ void run(float2* a) {
        float2 t = a[1];
        a[1] = csub(a[0], t);
        a[0] = cadd(a[0], t);
    }
};

template <int DIR>
struct DFT<4, DIR> {
    static __device__ __forceinline__ void run(float2* a) {
        float2 t0 = cadd(a[0], a[2]), t1 = csub(a[0], a[2]);
        float2 t2 = cadd(a[1], a[3]), t3 = mul_dir_i<DIR>(csub(a[1], a[3]));
        a[0] = cadd(t0, t2);
        a[2] = csub(t0, t2);
        a[1] = cadd(t1, t3);
        a[3] = csub(t1, t3);
    }
};

template <int DIR>
struct DFT<8, DIR> {
    // radix-2 split: even / odd halves as DFT4, twiddles exp(DIR 2 pi i k/8)
    static __device__ __forceinline__ void run(float2* a) {
        float2 e[4] = {a[0], a[2], a[4], a[6]};
        float2 o[4] = {a[1], a[3], a[5], a[7]};
        DFT<4, DIR>::run(e);
        DFT<4, DIR>::run(o);
        o[1] = rot16<DIR, 2>(o[1]);
        o[2] = rot16<DIR, 4>(o[2]);
        o[3] = rot16<DIR, 6>(o[3]);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            a[k] = cadd(e[k], o[k]);
            a[k + 4] = csub(e[k], o[k]);
        }
    }
};

template <int DIR>
struct DFT<16, DIR> {
    // 4 x 4 split: X[k1 + 4 k2] = sum_n2 w4^(n2 k2) w16^(n2 k1) sum_n1 a[4 n1 + n2] w4^(n1 k1)
    template <int N2>
    static __device__ __forceinline__ void col(float2* a, float2 (&b)[4][4]) {
        float2 t[4] = {a[N2], a[N2 + 4], a[N2 + 8], a[N2 + 12]};
        DFT<4, DIR>::run(t);
        b[N2][0] = t[0];
        b[N2][1] = rot16<DIR, N2 * 1>(t[1]);
        b[N2][2] = rot16<DIR, N2 * 2>(t[2]);
        b[N2][3] = rot16<DIR, N2 * 3>(t[3]);
    }
    static __device__ __forceinline__ void run(float2* a) {
        float2 b[4][4];
        col<0>(a, b);
        col<1>(a, b);
        col<2>(a, b);
        col<3>(a, b);
#pragma unroll
        for (int k1 = 0; k1 < 4; ++k1) {
            float2 t[4] = {b[0][k1], b[1][k1], b[2][k1], b[3][k1]};
            DFT<4, DIR>::run(t);
#pragma unroll
            for (int k2 = 0; k2 < 4; ++k2) a[k1 + 4 * k2] = t[k2];
        }
    }
};

// ------------------------------------------------------------ global access
// The step kernels read their array pointers from a table in device memory,
// so the compiler sees generic pointers and would emit FLAT loads and stores
// (which also hold the LDS counter).  Every such array is device memory:
// access it through global (address space 1) pointers, 8 bytes at a time.
typedef __attribute__((address_space(1))) double pss_gdouble;
typedef __attribute__((address_space(1))) uint64_t pss_gu64;
__device__ __forceinline__ float2 gload(const float2* p) {
    const pss_gdouble* q = (const pss_gdouble*)(p);
    return __builtin_bit_cast(float2, *q);
}
__device__ __forceinline__ void gstore(float2* p, float2 v) {
    pss_gdouble* q = (pss_gdouble*)(p);
    *q = __builtin_bit_cast(double, v);
}
__device__ __forceinline__ uint64_t gload_u64(const uint64_t* p) { return *(const pss_gu64*)(p); }
// A store marked non-temporal (NT): the line is not kept dirty in this XCD's
// L2, so the kernel's end has less to write back.  The step kernels of one
// lattice store this way (the next kernel reads the array from other XCDs);
// batched launches measured faster with plain stores.
template <bool NT>
__device__ __forceinline__ void gstore_sel(float2* p, float2 v) {
    pss_gdouble* q = (pss_gdouble*)(p);
    if constexpr (NT) {
        __builtin_nontemporal_store(__builtin_bit_cast(double, v), q);
    } else {
        *q = __builtin_bit_cast(double, v);
    }
}
// two neighbouring float2 in one 16-byte load (p 16-byte aligned).  Loaded
// as four floats: the same load typed as two doubles and split by bit casts
// compiled here to overlapping destination registers for loads in flight,
// which dropped the second element (caught by the parity tests)
typedef float pss_fvec4 __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(1))) pss_fvec4 pss_gfvec4;
__device__ __forceinline__ void gload_pair(const float2* p, float2& a, float2& b) {
    const pss_fvec4 v = *(const pss_gfvec4*)(p);
    a = make_float2(v.x, v.y);
    b = make_float2(v.z, v.w);
}

// ------------------------------------------------------------ block order
// The hardware hands out the blocks of a grid round-robin over the 8 XCDs
// (block b starts on XCD b mod 8), and each XCD has its own L2.  Renumber
// the blocks so that every XCD works on one contiguous range of logical
// blocks: neighbouring rows or lines that share cache lines then share an
// L2.  A bijection on [0, n) for any n.
__device__ __forceinline__ int xcd_block(int b, int n) {
    constexpr int X = 8;
    const int per = n / X, rem = n % X;
    const int x = b % X, k = b / X;
    return (x < rem ? x * (per + 1) : rem * (per + 1) + (x - rem) * per) + k;
}

// ------------------------------------------------------------------ Philox
#define PSS_PHILOX_M0 0xD2511F53u
#define PSS_PHILOX_M1 0xCD9E8D57u
#define PSS_PHILOX_W0 0x9E3779B9u
#define PSS_PHILOX_W1 0xBB67AE85u

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int i = 0; i < 10; ++i) {
        if (i) {
            k0 += PSS_PHILOX_W0;
            k1 += PSS_PHILOX_W1;
        }
        // 32 x 32 -> 64-bit products: one multiply gives both halves
        const uint64_t p0 = static_cast<uint64_t>(PSS_PHILOX_M0) * c.x;
        const uint64_t p1 = static_cast<uint64_t>(PSS_PHILOX_M1) * c.z;
        const uint32_t hi0 = static_cast<uint32_t>(p0 >> 32), lo0 = static_cast<uint32_t>(p0);
        const uint32_t hi1 = static_cast<uint32_t>(p1 >> 32), lo1 = static_cast<uint32_t>(p1);
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    }
    return c;
}

// (floor(w / 2^9) + 1/2) 2^-23: exact in binary32, inside (0, 1)
__device__ __forceinline__ float uniform23(uint32_t w) {
    return (static_cast<float>(w >> 9) + 0.5f) * 1.1920928955078125e-07f;
}

// Two standard normals from the first two words (Box & Muller 1958), with
// the hardware transcendentals: v_log_f32 (log2), v_sqrt_f32, and
// v_sin_f32 / v_cos_f32, whose argument is in revolutions (sin(2 pi u)).
__device__ __forceinline__ float2 box_muller(uint32_t w0, uint32_t w1) {
    const float u0 = uniform23(w0), u1 = uniform23(w1);
    // -2 ln u0 = -2 ln2 log2 u0 >= 0; clamp the rounding of log2 near u0 = 1
    const float r = __builtin_amdgcn_sqrtf(fmaxf(-1.3862943611198906f * __builtin_amdgcn_logf(u0), 0.f));
    return make_float2(r * __builtin_amdgcn_cosf(u1), r * __builtin_amdgcn_sinf(u1));
}

}  // namespace pss
