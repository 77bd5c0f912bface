// Line transforms for gfx950: a line of L complex points is held by T = L/P
// consecutive threads, P points each, and transformed by the recursive
// Cooley-Tukey splitting L = R * (L/R) (C. Van Loan, "Computational
// Frameworks for the Fast Fourier Transform", SIAM 1992, Sec. 1.3 and 2.1).
//
// Decimation in frequency (dif): thread t holds x[t + m T] in v[m] on entry.
// A stage over a sub-transform of length Ls, held by a group of G = Ls/P
// threads (thread g of the group holds element g + j G in v[j]), writes
// n = n1 (Ls/R) + n2, takes the R-point DFTs over n1 in registers, multiplies
// by the twiddles w_Ls^(n2 k1), and hands sub-transform k1 (length Ls/R) to
// the k1-th subgroup of G/R threads through LDS.  The first radix is
// L / P^s (1 if L is a power of P), every later one is P.  The last stage
// (G = 1) leaves X[D(t) + m T] in v[m], where D(t) collects the subgroup
// indices of t (a digit reversal).
//
// Decimation in time (dit) runs the same stages backwards: it takes
// X[D(t) + m T] in v[m] and leaves x[t + m T], natural order.  Both compute
// the unnormalised transform of sign DIR (-1 forward, +1 inverse).
//
// Callers gather their input from, or scatter their output to, global memory
// at the positions D(t) + m T, so the registers of the update step stay in
// natural mode order and no exchange is spent on reordering.
//
// Only a group spanning more than one wave (the first stage of a line of
// more than 64 threads) exchanges across waves, with one block barrier.  All
// other exchanges stay inside a wave: LDS performs one wave's operations in
// issue order, so they need no barrier, only a compiler-level ordering.
//
// LDS per line (LineFFT::kLds elements): a region for the in-wave exchanges
// (each group writes only its own Ls elements) and, for lines wider than a
// wave, two buffers for the block exchanges, used alternately (LdsLine::par):
// a buffer is written again only after the next block barrier, which every
// thread reaches after it has read the older exchange.  Each region holds
// kReg = L + L/2^PSS_FFT_PAD elements: element e of an exchange sits at
// e + (e >> PSS_FFT_PAD), one pad slot after every 2^PSS_FFT_PAD elements,
// so that the strided exchange patterns spread over the LDS banks (lines of
// 4096 stay unpadded, see pss_fft_layout.h).
#pragma once

#include "pss_device.h"
#include "pss_fft_layout.h"

namespace pss {

__host__ __device__ constexpr int first_radix(int L, int P) {
    int M = 1;
    while (M * P <= L) M *= P;
    return L / M;
}

// compiler-level ordering of the LDS accesses of one wave (no instruction)
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// LDS of one line: in-wave region and the two block-exchange buffers
struct LdsLine {
    float2* wl;
    float2* blk0;
    float2* blk1;
    int par;  // block buffer of the next block exchange (0 or 1)
    __device__ __forceinline__ float2* next_blk() {
        float2* b = par ? blk1 : blk0;
        par ^= 1;
        return b;
    }
};

template <int L, int P, int PADS = kFftPad>
struct LineFFT {
    static_assert((L & (L - 1)) == 0 && (P & (P - 1)) == 0 && P <= 16 && P <= L, "bad line shape");
    static constexpr int T = L / P;
    static constexpr bool kCross = T > 64;                  // the first exchange crosses waves
    static constexpr int kReg = fft_region(L, PADS);        // one exchange region
    static constexpr int kLds = kCross ? 3 * kReg : kReg;  // LDS elements per line
    static __device__ __forceinline__ int pad(int e) { return fft_padded(L, PADS) ? e + (e >> PADS) : e; }

    // stage s: sub-transform length, group size and radix
    struct Stages {
        int n;
        int Ls[16], G[16], R[16];
    };
    static constexpr Stages stages() {
        Stages st{};
        int Ls = L, G = T, R = first_radix(L, P) > 1 ? first_radix(L, P) : P;
        st.n = 0;
        while (true) {
            st.Ls[st.n] = Ls;
            st.G[st.n] = G;
            st.R[st.n] = R;
            ++st.n;
            if (Ls == R) break;
            Ls /= R;
            G /= R;
            R = P;
        }
        return st;
    }
    static constexpr Stages kSt = stages();

    // D(t): the first output index held by thread t after dif
    template <int S>
    static __device__ __forceinline__ void drev_acc(int& d, int& mul, int& g) {
        if constexpr (S < kSt.n) {
            constexpr int G = kSt.G[S], R = kSt.R[S];
            if constexpr (G > 1) {
                constexpr int Gn = G / R;
                d += mul * (g / Gn);
                mul *= R;
                g &= Gn - 1;
            }
            drev_acc<S + 1>(d, mul, g);
        }
    }
    static __device__ __forceinline__ int drev(int t) {
        int d = 0, mul = 1, g = t;
        drev_acc<0>(d, mul, g);
        return d;
    }

    template <int DIR>
    static __device__ __forceinline__ float2 twiddle(const float2* __restrict__ tw, int i) {
        float2 w = tw[i];
        if (DIR > 0) w.y = -w.y;
        return w;
    }

    template <int DIR, int S>
    static __device__ __forceinline__ void dif_stage(float2 (&v)[P], LdsLine& ld, int t,
                                                     const float2* __restrict__ tw) {
        constexpr int Ls = kSt.Ls[S], G = kSt.G[S], R = kSt.R[S];
        constexpr int PR = P / R;
        const int g = t & (G - 1);
#pragma unroll
        for (int h = 0; h < PR; ++h) {
            float2 a[R];
#pragma unroll
            for (int i = 0; i < R; ++i) a[i] = v[h + i * PR];
            DFT<R, DIR>::run(a);
            if constexpr (Ls > R) {
                const int n2 = g + h * G;
#pragma unroll
                for (int k1 = 1; k1 < R; ++k1) a[k1] = cmul(a[k1], twiddle<DIR>(tw, n2 * k1 * (L / Ls)));
            }
#pragma unroll
            for (int k1 = 0; k1 < R; ++k1) v[h + k1 * PR] = a[k1];
        }
        if constexpr (Ls > R) {
            constexpr int Gn = G / R;
            constexpr int Lr = Ls / R;
            constexpr bool cross = G > 64;
            float2* __restrict__ buf = cross ? ld.next_blk() : ld.wl;
            const int gb = (t - g) * P;  // the group's Ls elements
            if constexpr (!cross) wave_lds_sync();
#pragma unroll
            for (int h = 0; h < PR; ++h)
#pragma unroll
                for (int k1 = 0; k1 < R; ++k1) buf[pad(gb + k1 * Lr + g + h * G)] = v[h + k1 * PR];
            if constexpr (cross) {
                __syncthreads();
            } else {
                wave_lds_sync();
            }
            const int k1 = g / Gn, gp = g & (Gn - 1);
#pragma unroll
            for (int j = 0; j < P; ++j) v[j] = buf[pad(gb + k1 * Lr + gp + j * Gn)];
            dif_stage<DIR, S + 1>(v, ld, t, tw);
        }
    }

    template <int DIR, int S>
    static __device__ __forceinline__ void dit_stage(float2 (&v)[P], LdsLine& ld, int t,
                                                     const float2* __restrict__ tw) {
        constexpr int Ls = kSt.Ls[S], G = kSt.G[S], R = kSt.R[S];
        constexpr int PR = P / R;
        const int g = t & (G - 1);
        if constexpr (Ls > R) {
            dit_stage<DIR, S + 1>(v, ld, t, tw);
            constexpr int Gn = G / R;
            constexpr int Lr = Ls / R;
            constexpr bool cross = G > 64;
            float2* __restrict__ buf = cross ? ld.next_blk() : ld.wl;
            const int gb = (t - g) * P;
            const int k1 = g / Gn, gp = g & (Gn - 1);
            if constexpr (!cross) wave_lds_sync();
#pragma unroll
            for (int j = 0; j < P; ++j) buf[pad(gb + k1 * Lr + gp + j * Gn)] = v[j];
            if constexpr (cross) {
                __syncthreads();
            } else {
                wave_lds_sync();
            }
#pragma unroll
            for (int h = 0; h < PR; ++h)
#pragma unroll
                for (int kk = 0; kk < R; ++kk) v[h + kk * PR] = buf[pad(gb + kk * Lr + g + h * G)];
        }
#pragma unroll
        for (int h = 0; h < PR; ++h) {
            float2 a[R];
#pragma unroll
            for (int k1 = 0; k1 < R; ++k1) a[k1] = v[h + k1 * PR];
            if constexpr (Ls > R) {
                const int n2 = g + h * G;
#pragma unroll
                for (int k1 = 1; k1 < R; ++k1) a[k1] = cmul(a[k1], twiddle<DIR>(tw, n2 * k1 * (L / Ls)));
            }
            DFT<R, DIR>::run(a);
#pragma unroll
            for (int i = 0; i < R; ++i) v[h + i * PR] = a[i];
        }
    }

    // natural order in, X[D(t) + m T] out
    template <int DIR>
    static __device__ __forceinline__ void dif(float2 (&v)[P], LdsLine& ld, int t, const float2* __restrict__ tw) {
        dif_stage<DIR, 0>(v, ld, t, tw);
    }
    // X[D(t) + m T] in, natural order out
    template <int DIR>
    static __device__ __forceinline__ void dit(float2 (&v)[P], LdsLine& ld, int t, const float2* __restrict__ tw) {
        dit_stage<DIR, 0>(v, ld, t, tw);
    }
};


}  // namespace pss
