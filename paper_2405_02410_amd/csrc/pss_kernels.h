// Launch interface between the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "pss_fft_layout.h"
#include "pss_plan.h"

namespace pss {

// kernel modes
enum {
    MODE_STEP = 0,       // one time step
    MODE_PROLOGUE = 1,   // update kernel: masked inverse of the current state only
    MODE_FWD_STORE = 2,  // update kernel: forward transform of `in`, stored as state `sel`
    MODE_INV_OUT = 3,    // update kernel: inverse transform of state `sel` into `out`
    MODE_R2C_IN = 4,     // x kernel: real rows `real_in` -> packed columns `out`
    MODE_C2R_OUT = 5,    // x kernel: packed columns `in` -> real rows `real_out`
    MODE_YINV = 6,       // y pass (3D): inverse transform, column-0 slots -> packed
    MODE_YFWD = 7,       // y pass (3D): forward transform, column-0 packed -> slots
    MODE_ADJROW = 8,     // x kernel: adjoint row pass (Model B), see AdjArgs
    MODE_ADJCOL = 9,     // adjoint column kernel: one reverse step
    MODE_ADJFIN = 10,    // adjoint column kernel: g_0 from the last reverse step
    MODE_INTERM_OUT = 11,  // update kernel: inverse transform of intermediate `sel` into `out`
};

// Device arrays used by a launch (all in the packed half-spectrum layout
// except the real-space ones).
struct Bufs {
    float2* S[PSS_MAXF];   // state per field
    float2* N[PSS_MAXCH];  // product channels (x kernel writes, update kernel reads)
    float2* V[PSS_MAXG];   // de-aliased inverse transforms per factor slot
    const float2* in;
    float2* out;
    const float* real_in;
    float* real_out;
    double* acc;  // adjoint row pass: one FP64 slot per block of sum_x u^3 w
    int sel;
};

// Reverse step of 2D Model B (phi_{n+1} = (phi_n + dt M F[u_n^3] + eta_n) / A,
// u_n = Re F^-1[m phi_n], M = -b q^2, A = 1 + dt q^2 (a + k q^2)), adjoint
// column kernel.  All spectral arrays are packed, in the 2D state layout.
//   g_{n+1} = first ? G : Rin + b m F_y[X] / N    (X: x-forward of 3 u^2 w, row pass)
//   r_n = g_{n+1} / A                             -> Rout
//   dL/da -= <r, dt q^2 phi1>, dL/dk -= <r, dt q^4 phi1>, dL/dD += <r, eta_n>/(2D)
//   W = F_y^-1[-dt q^2 r_n],  U = F_y^-1[m phi0]
// The row pass (x kernel, MODE_ADJROW) forms w = N F^-1[-dt q^2 r_n] and
// u_n in real space and adds <r, -dt q^2 F[u_n^3]> = sum_x u^3 w to dL/db,
// with <x, y> = Re sum over all modes of conj(x) y.  Each block adds its part
// of a sum into slots of its own (the same blocks every step), which the host
// sums in a fixed order after the sweep.  MODE_ADJFIN stops after g_{n+1} and
// stores it in Rout.
struct AdjArgs {
    const DevPlan* plan;  // forward plan: masks, noise operator, q scales, keys
    const float2* G;
    const float2* Rin;
    const float2* X;
    const float2* phi1;   // phi_{n+1}
    const float2* phi0;   // phi_n
    float2* Rout;
    float2* W;
    float2* U;
    double* acc;          // [3 * blocks]: per block dL/da, dL/dk, dL/dD
    float a, b, k, D;
    uint32_t step;        // n: the noise counter of the forward step
    int first;
};

struct Geo {
    int tc;       // packed columns per tile
    int rb;       // rows per x-kernel block (even)
    int ntile;    // tiles (= Nx/2 / tc)
    int nrowblk;  // x-kernel blocks (= rows / rb)
    int to;       // update kernel: other-index lines per block (3D: y values; 2D: 1)
    int nublk;    // update-kernel blocks (= ntile * Ny/to in 3D, ntile in 2D)
    int tz;       // y pass: z values per block
    int nyblk;    // y-pass blocks (= ntile * Nz/tz)
    int nz;       // Nz (1 in 2D)
    int tc_log2;  // log2(tc)
    int rb_log2;  // log2(rb)
    int pu;       // points per thread: update kernel
    int px;       // points per thread: x kernel
    int py;       // points per thread: y pass
};

// arrays handled by one y-pass launch
struct YArgs {
    const float2* src[PSS_MAXCH];
    float2* dst[PSS_MAXCH];
    int ncol[PSS_MAXCH];  // only tiles with columns below ncol are transformed
    int n;
};

// One lattice of a step launch.  The step kernels (update STEP / PROLOGUE,
// x STEP) read buffers and step counter of lattice blockIdx.y from a table of
// these in device memory, and its plan from a parallel array of plans (a
// kernel argument of its own, so that the plan reads are scalar loads); the
// lattices of one launch share the geometry (sizes, fields, factors,
// channels, tiling) and the twiddles.
struct Member {
    Bufs bufs;
    uint64_t* step_ctr;
    uint32_t* flag;  // bit f set when a non-finite value appears in field f's new state
};

struct LaunchArgs {
    hipStream_t stream;
    const DevPlan* plan;
    Bufs bufs;
    Geo geo;
    const uint64_t* step_ctr;
    uint32_t* flag;         // the non-finite flag of the single lattice (transform modes)
    const Member* members;  // step modes: table of nmem lattices (device memory)
    const DevPlan* plans;   // step modes: their nmem plans (device memory)
    int nmem;
    bool general;           // the plans need the general-monomial operator code
    int step_off;
    int64_t advance;     // x kernel, step modes: add this to every member's step counter (0: none)
    const float2* tw_u;  // twiddles of the update-axis length
    const float2* tw_x;  // twiddles of Nx
    const float2* tw_y;  // twiddles of Ny (3D y passes)
    int dim;             // 1, 2 or 3
    int nsteps;          // 1D step launches: steps of the launch
    int ng;              // factor slots of the plan (1D lines of mixed-radix length size their LDS by it)
    int nx, ny, nz;      // lattice sizes (the mixed-radix launches)
};

// Fused batch launches: one update-phase and one x-phase launch cover every
// size class of a batch whose lattices fit the fused kernels (2D, one field,
// 4 points per thread, 256-thread blocks, lines of 64 .. 1024).  Blocks are a
// work list of (class, member, tile): class k owns blocks [start, start +
// nmem * nblk), member-major.
constexpr int kMaxBatchClasses = 8;
struct BatchClass {
    int L;      // line length of the phase (update: Ny; x: Nx)
    int start;  // first block of the class
    int nblk;   // blocks per member
    int pad;
    const Member* members;
    const DevPlan* plans;
    const float2* tw;  // twiddles of L
    Geo geo;           // the class's launch geometry for this phase
};
struct BatchLaunch {
    int ncls;      // classes in the launch
    int total;     // blocks
    int step_off;  // step within the replayed chunk (update phase)
    int pad;
    int64_t advance;  // x phase: counter advance of the chunk's last step (0: none)
    BatchClass cls[kMaxBatchClasses];
};
// line lengths the fused kernels are built for
inline bool batch_fused_len(int L) { return L >= 64 && L <= 1024 && (L & (L - 1)) == 0; }

// LDS-resident launch: lattices whose whole packed half spectrum and channel
// array fit in one CU's LDS take many steps in one launch, one block per
// member, with no HBM traffic between steps (2D, Nx and Ny in {64, 128}; one
// field whose real-space products use that field only; 4 points per thread
// in both phases, as the per-lattice kernels use them, so the arithmetic and
// its rounding are the same).
struct ResidentLaunch {
    int lx, ly;   // lattice sizes
    int nmem;     // members (blocks)
    int nsteps;   // steps of the launch
    int advance;  // 1: the launch moves the members' step counters on by nsteps
    int pad;
    const Member* members;  // update-kernel table: state S[0], channel N[0], counter, flag
    const DevPlan* plans;
    const float2* tw_x;  // twiddles of Nx and of Ny
    const float2* tw_y;
    Geo geo;  // tc, tc_log2: the global layout of S and N
};
__host__ __device__ constexpr int resident_threads(int lx, int ly) {
    return (lx / 2) * (ly / 4) < 1024 ? (lx / 2) * (ly / 4) : 1024;
}
// LDS: padded channel/factor array, line scratch, packed-line exchange, twiddles
inline size_t resident_lds_bytes(int lx, int ly) {
    const int nthr = resident_threads(lx, ly);
    const size_t scr_y = static_cast<size_t>(nthr / (ly / 4)) * fft_region(ly);
    const size_t scr_x = static_cast<size_t>(nthr / (lx / 4)) * fft_region(lx);
    return sizeof(float2) * (static_cast<size_t>(lx / 2) * (ly + 1) + (scr_y > scr_x ? scr_y : scr_x) + 2 * ly + lx);
}
inline bool resident_shape(int lx, int ly) { return (lx == 64 || lx == 128) && (ly == 64 || ly == 128); }
hipError_t resident_setup();
hipError_t launch_batch_resident(hipStream_t s, const ResidentLaunch& rl);
hipError_t launch_batch_update(hipStream_t s, const BatchLaunch& bl, size_t lds);
hipError_t launch_batch_xrow(hipStream_t s, const BatchLaunch& bl, size_t lds);

// largest points per thread a kernel is built for with `nregs` register
// arrays of fields (1, 2 or 4 and more): 16, 8, 4, capped at L
int max_points(int L, int nregs);

hipError_t launch_update(int mode, int L, int nf, const LaunchArgs& a);

// 1D lattices: one block holds the whole line (line1d_kernel).  Modes:
// MODE_STEP (a.nsteps steps; a.advance != 0 moves the counter on by them),
// MODE_FWD_STORE (real_in -> state sel), MODE_INV_OUT (state sel ->
// real_out), MODE_INTERM_OUT (intermediate sel -> real_out).  The state of a
// field is its full complex spectrum of N modes in natural order.
hipError_t launch_line1d(int mode, int N, int nf, const LaunchArgs& a);
// LDS of the 1D kernel: the line transform, the twiddle table and a
// real-space staging line for the boundary frames
inline size_t line1d_lds_bytes(int N) {
    return sizeof(float2) * (static_cast<size_t>(fft_lds_elems(N, 4, 1)) + static_cast<size_t>(N)) +
           sizeof(float) * static_cast<size_t>(N);
}
// allow the 1D kernels of length N their LDS (above the default dynamic limit)
hipError_t line1d_setup(int N);

// 1D lines of mixed-radix length N = 2^a 3^b 5^c, a >= 1, not a power of two
// (launch_line1d sends them to their own kernel): the radices of the
// self-sorting passes, 4 first, then 2, 3 and 5.  False if N does not factor
// so or is not even.
struct MrPlan {
    int n;
    int nst;
    int radix[24];
};
inline bool mr_plan(int N, MrPlan* mr) {
    if (N < 2 || (N & 1)) return false;
    mr->n = N;
    mr->nst = 0;
    int n = N;
    while (n % 4 == 0 && n > 4) {
        mr->radix[mr->nst++] = 4;
        n /= 4;
    }
    for (int r : {4, 2, 3, 5})
        while (n % r == 0) {
            if (mr->nst >= 24) return false;
            mr->radix[mr->nst++] = r;
            n /= r;
        }
    return n == 1;
}
// LDS of the mixed-radix 1D kernel: twiddle table, two transform buffers,
// NF states and NF contribution arrays (complex), ng real factor lines
inline size_t line1d_mr_lds_bytes(int N, int NF, int ng) {
    return sizeof(float2) * static_cast<size_t>(N) * (3 + 2 * static_cast<size_t>(NF)) +
           sizeof(float) * static_cast<size_t>(N) * static_cast<size_t>(ng > 0 ? ng : 1);
}
hipError_t launch_line1d_mr(int mode, int N, int nf, int ng, const LaunchArgs& a);
hipError_t line1d_mr_setup();

// 2D and 3D lattices of mixed-radix sizes (even 2^a 3^b 5^c, not all powers
// of two): full complex spectra, mode (kx, ky, kz) at (kz Ny + ky) Nx + kx.  Column launch
// (geo.tc neighbouring lines per block): MODE_STEP (channels N[ch] in (y, kx) form -> update ->
// factors V[g] in (y, kx) form), MODE_PROLOGUE (factors from the state),
// MODE_FWD_STORE (in, (y, kx) -> state sel), MODE_INV_OUT (state sel -> out,
// (y, kx)), MODE_INTERM_OUT (intermediate sel -> out).  Row launch (one block
// per y): MODE_STEP (V -> products -> N; a.advance moves the counter on),
// MODE_R2C_IN (real_in -> out), MODE_C2R_OUT (in -> real_out, normalised).
// column launch: the twiddles of a line, then two transform buffers, NF
// states and NF contribution arrays of tc lines each; the y pass: the
// twiddles and two buffers of tc lines
inline size_t mr2_col_lds_bytes(int L, int NF, int tc) {
    return sizeof(float2) * static_cast<size_t>(L) * (1 + static_cast<size_t>(tc) * (2 + 2 * static_cast<size_t>(NF)));
}
inline size_t mr3_ypass_lds_bytes(int Ny, int tc) {
    return sizeof(float2) * static_cast<size_t>(Ny) * (1 + 2 * static_cast<size_t>(tc));
}
inline size_t mr2_row_lds_bytes(int Nx, int ng) {
    return sizeof(float2) * static_cast<size_t>(Nx) * 3 +
           sizeof(float) * static_cast<size_t>(Nx) * static_cast<size_t>(ng > 0 ? ng : 1);
}
// In 3D the column launch runs along z (geo.tc lines of neighbouring kx per
// block), the row launch covers Ny Nz rows, and launch_mr3_ypass transforms
// the arrays of ya along y (sign -1 forward, +1 inverse), geo.py lines of
// neighbouring kx per block.
hipError_t launch_mr2_col(int mode, int nf, const LaunchArgs& a);
hipError_t launch_mr2_row(int mode, const LaunchArgs& a);
hipError_t launch_mr3_ypass(int sign, const YArgs& ya, const LaunchArgs& a);
hipError_t mr2_setup();
hipError_t launch_xrow(int mode, int L, int ng, const LaunchArgs& a);
hipError_t launch_ypass(int mode, int L, const YArgs& ya, const LaunchArgs& a);
hipError_t launch_advance(hipStream_t s, uint64_t* step_ctr, int64_t k);
// adjoint column kernel (2D, one field) and its launch
hipError_t launch_adjcol(int mode, int L, const AdjArgs& aa, const LaunchArgs& a);
// terminal seed g = coef[shell(k)] * phi (2D packed state layout)
hipError_t launch_adjseed(hipStream_t s, const float2* phi, float2* g, const float* coef, int nshell, int nx, int ny,
                          int tc);

// *ctrs[i] += k for i < n (the step counters of a batch)
hipError_t launch_advance_many(hipStream_t s, uint64_t* const* ctrs, int n, int64_t k);
// out[i] = the non-finite flag word after *ctrs[i] (the word after the step
// counter), cleared atomically
hipError_t launch_take_flags(hipStream_t s, uint64_t* const* ctrs, int n, uint32_t* out);
// real[frame[i].x] = value bits frame[i].y, i < n (a boundary frame on a real-space array)
hipError_t launch_apply_frame(hipStream_t s, float* real, const int2* frame, int n);
hipError_t launch_init_uniform(hipStream_t s, float* out, int64_t n, uint32_t field, uint32_t key0, uint32_t key1,
                               double lo, double hi);
hipError_t launch_philox(hipStream_t s, uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                         int64_t count, uint32_t* out);

// register-array count an instantiation is built for (1, 2 or 4 fields)
inline int field_slots(int n) { return n <= 1 ? 1 : (n == 2 ? 2 : 4); }
// LDS elements of the line transforms of `lines` lines of length L held with
// P points per thread: one in-wave region per line, plus two block-exchange
// buffers per line when a line spans more than one wave (pss_fft.h)
inline size_t fft_lds(int L, int P, int lines, int pads = kFftPad) {
    return static_cast<size_t>(fft_lds_elems(L, P, lines, pads));
}
// dynamic LDS of the update kernel: TC*TO line transforms, one exchange line
// and the staged twiddle table (L entries), in that order
inline size_t update_lds_bytes(int L, int P, int tc, int to, int pads = kFftPad) {
    return sizeof(float2) * (fft_lds(L, P, tc * to, pads) + 2 * static_cast<size_t>(L));
}
// dynamic LDS of the y pass: TC*TZ line transforms, one exchange line per z
// and the staged twiddle table (L entries), in that order
inline size_t ypass_lds_bytes(int L, int P, int tc, int tz) {
    return sizeof(float2) * (fft_lds(L, P, tc * tz) + static_cast<size_t>(tz + 1) * L);
}
// dynamic LDS of the x kernel: RB/2 line transforms + the staged twiddle table
inline size_t xrow_lds_bytes(int L, int P, int rb) {
    return sizeof(float2) * (fft_lds(L, P, rb / 2) + static_cast<size_t>(L));
}

// Allocation-free reductions (pss_noalloc.hip): the device address of the
// file-scope scratch array on the current device, looked up once per device,
// and a fill kernel that clears n 64-bit words of it
constexpr int kScratchShells = 2048;
hipError_t scratch_address(void** out);
hipError_t launch_zero_words(hipStream_t s, unsigned long long* p, int n);

// Shell means of (dV/N)|phi_hat|^2 over the packed state of one field, from
// exact fixed-point sums (the result does not depend on the order of the
// atomics).  acc holds kShellWords * nshell zeroed 64-bit words; on return
// acc[j] holds the mean of shell j as a double and acc[2 * nshell + j] its
// population.
constexpr int kShellWords = 4;
hipError_t launch_shells(hipStream_t s, const float2* S, int nx, int ny, int nz, int tc, int ndim,
                         double scale, int nshell, unsigned long long* acc);


}  // namespace pss
