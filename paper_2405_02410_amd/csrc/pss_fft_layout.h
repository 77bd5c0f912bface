// LDS sizes of the line transforms (pss_fft.h), shared with the host code
// that sizes the kernels' dynamic LDS.
#pragma once

// one pad element after every 2^PSS_FFT_PAD elements of an exchange region
#ifndef PSS_FFT_PAD
#define PSS_FFT_PAD 3
#endif

namespace pss {

// pad shift of the per-lattice kernels; 0 means no padding (the fused batch
// kernels, where the pad's address registers would cost occupancy)
constexpr int kFftPad = PSS_FFT_PAD;

// elements of one exchange region of a line of L points, padded by shift
// `pads`; lines of 4096 keep the unpadded layout, so that such a line with
// its packed-line exchange and twiddle table still fits in one workgroup's
// 160 KiB
constexpr bool fft_padded(int L, int pads) { return pads > 0 && L < 4096; }
constexpr int fft_region(int L, int pads = kFftPad) { return fft_padded(L, pads) ? L + (L >> pads) : L; }

// LDS elements of the line transforms of `lines` lines of L points held by
// L/P threads each: one region per line, three when a line spans waves
constexpr int fft_lds_elems(int L, int P, int lines, int pads = kFftPad) {
    return lines * ((L / P > 64) ? 3 : 1) * fft_region(L, pads);
}

}  // namespace pss
