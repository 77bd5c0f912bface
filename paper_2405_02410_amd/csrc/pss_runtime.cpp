// Host runtime behind include/pss.h: context, validation, plan compilation,
// device buffers, captured step graphs, state I/O and reductions.
//
// The model is the paper's term structure (eq:basereal): implicit operators
// build L(q) of each field; explicit single-factor linear terms act directly
// in Fourier space; every other explicit term is a product of de-aliased
// fields formed in real space.  Terms with the same target and the same single
// monomial operator shape share one real-space "channel" (their products are
// summed before the forward transform, which is linear).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cctype>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <numeric>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/pss.h"
#include "pss_error.h"
#include "pss_kernels.h"
#include "pss_plan.h"

namespace {
thread_local std::string g_err;
}  // namespace

// the message pss_last_error returns (also set by the equation front end)
pss_status pss_internal::set_error(pss_status code, const char* fmt, va_list ap) {
    char buf[512];
    vsnprintf(buf, sizeof(buf), fmt, ap);
    g_err = buf;
    return code;
}

namespace {

pss_status fail(pss_status code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    const pss_status s = pss_internal::set_error(code, fmt, ap);
    va_end(ap);
    return s;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t e_ = (expr);                                                              \
        if (e_ != hipSuccess) {                                                              \
            return fail(e_ == hipErrorOutOfMemory ? PSS_E_NOMEM : PSS_E_HIP, "%s: %s (%s:%d)", \
                        #expr, hipGetErrorString(e_), __FILE__, __LINE__);                     \
        }                                                                                    \
    } while (0)

struct Mono {
    double coef;
    int q2, invq, iq[3];
};

struct Term {
    int target;
    bool implicit;
    std::vector<Mono> op;
    std::vector<std::pair<int, int>> factors;  // (field, power)
    // where its coefficients live in the compiled plan
    int kind = 0;      // 0 implicit, 1 direct, 2 channel (single monomial), 3 channel (own operator),
                       // 4 a term of an intermediate field's equation
    int slot = -1;     // field / direct / channel index
    int mono0 = -1;    // first monomial index inside the slot operator (kinds 0, 1, 3)
    int prod = -1;     // product index inside the channel (kind 2)
};

struct Field {
    std::string name;
    bool noisy = false;
    std::vector<Mono> noise;
};

// Declared fields are numbered in declaration order.  Internally a dynamic
// field is its index among the dynamic fields and an intermediate field is
// PSS_MAXF + its index among the intermediates (the same codes the plan uses).
bool is_interm(int code) { return code >= PSS_MAXF; }

bool is_pow2(int64_t n) { return n > 0 && (n & (n - 1)) == 0; }

double op_real_at(const std::vector<Mono>& op, const double q[3], bool nyq[3], double* imag) {
    const double q2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2];
    const double invq = q2 > 0 ? 1.0 / std::sqrt(q2) : 0.0;
    double re = 0, im = 0;
    for (const Mono& m : op) {
        double s = m.coef * std::pow(q2, m.q2) * std::pow(invq, m.invq);
        int ip = 0;
        for (int i = 0; i < 3; ++i) {
            if (m.iq[i]) {
                s *= std::pow(nyq[i] ? 0.0 : q[i], m.iq[i]);
                ip += m.iq[i];
            }
        }
        switch (ip & 3) {
            case 0: re += s; break;
            case 1: im += s; break;
            case 2: re -= s; break;
            default: im -= s; break;
        }
    }
    if (imag) *imag = im;
    return re;
}

// FP32 twiddles exp(-2 pi i m / L), m = 0..L-1, computed in FP64 from the
// angle reduced to the first octant so every value is correctly rounded.
std::vector<float2> twiddles(int L) {
    std::vector<float2> w(L);
    for (int m = 0; m < L; ++m) {
        // angle = 2 pi m / L = (pi/4) * (8 m / L); split 8m = L*o + r
        const int64_t num = 8LL * m;
        const int oct = static_cast<int>(num / L);
        const double frac = static_cast<double>(num % L) / L;  // in [0, 1)
        // phase within the octant in units of pi/4
        double c, s;
        const double a = frac * (M_PI / 4);
        const double ca = std::cos(a), sa = std::sin(a);
        const double cb = std::cos(M_PI / 4 - a), sb = std::sin(M_PI / 4 - a);
        switch (oct & 7) {
            case 0: c = ca; s = sa; break;
            case 1: c = sb; s = cb; break;
            case 2: c = -sa; s = ca; break;
            case 3: c = -cb; s = sb; break;
            case 4: c = -ca; s = -sa; break;
            case 5: c = -sb; s = -cb; break;
            case 6: c = sa; s = -ca; break;
            default: c = cb; s = -sb; break;
        }
        w[m] = make_float2(static_cast<float>(c), static_cast<float>(-s));
    }
    return w;
}

}  // namespace

struct pss_ctx {
    int ndim = 2;
    bool mixed = false;  // 2D sizes that are not both powers of two: full spectra, mixed-radix kernels
    int n[3] = {1, 1, 1};
    double dx[3] = {1, 1, 1};
    double dt = 0;
    uint64_t seed = 0;
    int rule = PSS_DEALIAS_TWO_THIRDS, shape = PSS_SHAPE_RADIAL;
    std::vector<Field> fields;          // dynamic fields
    std::vector<std::string> interms;   // intermediate fields (names)
    std::vector<int> ids;               // declared field -> internal code
    std::vector<Term> terms;            // fields named by internal code
    std::vector<std::vector<int2>> frames;  // boundary frames per dynamic field: (site, value bits)
    std::map<std::string, double> params;   // named parameters of the equation front end

    // device side
    bool planned = false;
    bool dirty = true;  // channel arrays must be rebuilt from the state
    pss::DevPlan plan{};
    pss::Geo geo{};
    int lu = 0;  // update-axis length
    hipStream_t stream = nullptr;
    bool own_stream = false;
    pss::DevPlan* d_plan = nullptr;
    uint64_t* d_step = nullptr;
    float2* d_tw_u = nullptr;
    float2* d_tw_x = nullptr;
    float2* d_tw_y = nullptr;
    // d_chan: channel inputs of the update kernel; d_chan_x: x-kernel outputs
    // (the same arrays in 2D; in 3D the forward y pass maps one to the other)
    std::vector<float2*> d_state, d_chan, d_chan_x, d_v;
    void* bound[PSS_MAXF] = {};       // caller-owned state memory per dynamic field (pss_field_bind)
    size_t bound_bytes[PSS_MAXF] = {};
    float2* d_tmp = nullptr;
    float2* d_tmp2 = nullptr;
    float* d_real = nullptr;
    int2* d_frame[PSS_MAXF] = {};  // device copies of the frames
    unsigned long long* d_shell_acc = nullptr;  // shell accumulators (kShellWords per shell)
    // one-entry member tables of the step kernels (update kernel, x kernel)
    pss::Member* d_member_u = nullptr;
    pss::Member* d_member_x = nullptr;
    int batches = 0;        // live batches holding this context
    int tapes = 0;          // live adjoint tapes recorded on this context
    uint64_t state_gen = 0; // bumped by every change of the state (steps, uploads, loads)
    uint64_t enq_gen = 0;   // bumped whenever the context enqueues work on its own stream
    hipEvent_t after_batch = nullptr;  // the context's own work must wait for this batch event
    uint64_t plan_gen = 0;  // bumped at every upload of the plan
    std::map<int64_t, hipGraphExec_t> graphs;
    std::map<std::string, int64_t> tune;  // launch-geometry overrides
    int64_t steps_taken = 0;
    // PSS_DEBUG_SYNC set (and not "0") when the lattice was created: steps run
    // eagerly instead of as graphs, the stream is synchronised and checked
    // after every kernel, and the workspaces start filled with NaN
    bool debug_sync = false;

    int64_t sites() const { return static_cast<int64_t>(n[0]) * n[1] * n[2]; }
    // complex elements per spectral array: the packed half spectrum in 2D and
    // 3D, the full spectrum of the line in 1D
    int64_t packed() const { return ndim == 1 || mixed ? sites() : sites() / 2; }
};

// A set of 2D lattices stepped together.  Lattices with the same sizes,
// field / factor / channel counts and launch geometry form a class; each
// class runs as one update launch and one x launch per step, with the
// lattice picked by blockIdx.y from a device table of its plan, buffers and
// step counter.
struct pss_batch {
    struct Class {
        std::vector<int> idx;          // members of the class
        pss_ctx* rep = nullptr;        // first member: geometry and twiddles
        pss::Member* d_u = nullptr;    // member tables of the update and x kernels
        pss::Member* d_x = nullptr;
        pss::DevPlan* d_plans = nullptr;  // copies of the members' plans
        std::vector<uint64_t> gen;        // plan generation of each copy
    };
    std::vector<pss_ctx*> mem;
    std::vector<uint64_t> seen;        // members' enq_gen when the batch last ordered itself after them
    std::vector<int> all;              // 0 .. n-1
    std::vector<Class> cls;
    // fused launches: the classes that fit the fused kernels run in one
    // update-phase and one x-phase launch per step (templates; the step
    // offset and the counter advance are set per launch)
    pss::BatchLaunch fu{}, fx{};
    size_t fu_lds = 0, fx_lds = 0;
    std::vector<char> in_fu, in_fx;    // per class
    // LDS-resident classes: one launch per replayed chunk of steps
    std::vector<char> in_res;          // per class
    std::vector<pss::ResidentLaunch> res;
    bool resident = true;              // PSS_BATCH_RESIDENT=0 at creation turns the resident launches off
    uint64_t** d_ctrs = nullptr;       // step counter of every member
    uint32_t* d_flags = nullptr;       // the members' non-finite flags, gathered by pss_batch_sync
    hipStream_t stream = nullptr;      // the first member's stream
    hipEvent_t ev = nullptr;
    std::map<int64_t, hipGraphExec_t> graphs;
};

// Recorded forward run of the Model B adjoint: checkpoints of the state,
// the final state, the terminal-seed coefficients and the workspace of the
// reverse sweep, all owned by the tape until pss_tape_destroy.
struct pss_tape {
    pss_ctx* ctx = nullptr;
    std::vector<void*> mem;  // device allocations
    int64_t n0 = 0, nsteps = 0, nck = 0, seglen = 0;
    int32_t ckpt = 0, ns = 0;
    size_t fb = 0;  // bytes of one packed spectrum
    double a = 0, b = 0, k = 0, D = 0, loss = 0;
    uint64_t plan_gen = 0, state_gen = 0;
    bool done = false;  // the reverse sweep has run
    char* ck = nullptr;
    char* seg = nullptr;
    float2 *fT = nullptr, *G = nullptr, *R0 = nullptr, *R1 = nullptr, *X = nullptr, *W = nullptr, *U = nullptr;
    double* acc = nullptr;  // per-block FP64 slots of the gradient sums
    size_t nacc = 0;
    float* coef = nullptr;
    pss::DevPlan* plan_row = nullptr;
    pss::DevPlan* plan_raw = nullptr;
};

namespace {

int field_code(const pss_ctx* c, int32_t id) {
    return id >= 0 && id < static_cast<int32_t>(c->ids.size()) ? c->ids[id] : -1;
}

// a declared field that must be dynamic -> its dynamic index
pss_status dyn_field(const pss_ctx* c, int32_t id, int* f) {
    const int code = field_code(c, id);
    if (code < 0) return fail(PSS_E_INVAL, "bad field");
    if (is_interm(code)) return fail(PSS_E_INVAL, "field %d is an intermediate field, defined by its equation", id);
    *f = code;
    return PSS_OK;
}

pss_status check_ctx(pss_ctx* c) {
    if (!c) return fail(PSS_E_INVAL, "null context");
    return PSS_OK;
}

void* tape_alloc(pss_tape* tp, size_t bytes) {
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) return nullptr;
    tp->mem.push_back(p);
    return p;
}

void tape_free(pss_tape* tp) {
    if (tp->ctx && tp->ctx->stream) (void)hipStreamSynchronize(tp->ctx->stream);
    for (void* p : tp->mem) (void)hipFree(p);
    tp->mem.clear();
}

float2* tape_at(const pss_tape* tp, char* base, int64_t i) {
    return reinterpret_cast<float2*>(base + tp->fb * static_cast<size_t>(i));
}

pss_status check_ops(const pss_qmono* op, int32_t n_mono, bool noise) {
    if (n_mono < 1 || n_mono > PSS_MAXM) return fail(PSS_E_INVAL, "operator needs 1..%d monomials", PSS_MAXM);
    if (!op) return fail(PSS_E_INVAL, "null operator");
    for (int i = 0; i < n_mono; ++i) {
        const pss_qmono& m = op[i];
        if (!std::isfinite(m.coef)) return fail(PSS_E_INVAL, "non-finite coefficient");
        if (m.q2_pow < 0 || m.q2_pow > PSS_MAXPOW || m.invq_pow < 0 || m.invq_pow > PSS_MAXPOW)
            return fail(PSS_E_INVAL, "operator powers must lie in [0, %d]", PSS_MAXPOW);
        for (int k = 0; k < 3; ++k)
            if (m.iq_pow[k] < 0 || m.iq_pow[k] > PSS_MAXPOW)
                return fail(PSS_E_INVAL, "operator powers must lie in [0, %d]", PSS_MAXPOW);
        if (noise && (m.iq_pow[0] || m.iq_pow[1] || m.iq_pow[2]))
            return fail(PSS_E_INVAL, "a noise operator takes powers of q^2 and 1/|q| only");
    }
    return PSS_OK;
}

std::vector<Mono> to_monos(const pss_qmono* op, int n) {
    std::vector<Mono> v;
    for (int i = 0; i < n; ++i)
        v.push_back({op[i].coef, op[i].q2_pow, op[i].invq_pow, {op[i].iq_pow[0], op[i].iq_pow[1], op[i].iq_pow[2]}});
    return v;
}

// Visit every mode of the full spectrum with its q vector (FP64).
template <class F>
void for_each_mode(const pss_ctx* c, F&& fn) {
    const int nz = c->ndim == 3 ? c->n[2] : 1;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < c->n[1]; ++y)
            for (int x = 0; x <= c->n[0] / 2; ++x) {
                const int ny = c->n[1];
                const int k[3] = {x == c->n[0] / 2 ? -x : x, ny == 1 ? 0 : (y < ny / 2 ? y : y - ny),
                                  nz == 1 ? 0 : (z < nz / 2 ? z : z - nz)};
                double q[3];
                bool nyq[3];
                for (int i = 0; i < 3; ++i) {
                    const int ni = i < 2 ? c->n[i] : nz;
                    q[i] = 2 * M_PI * k[i] / (ni * c->dx[i]);
                    nyq[i] = ni > 1 && k[i] == -(ni / 2);
                }
                fn(q, nyq);
            }
}

pss_status validate(pss_ctx* c) {
    const int nf = static_cast<int>(c->fields.size());
    if (nf == 0) return fail(PSS_E_STATE, "no fields declared");
    const int ni = static_cast<int>(c->interms.size());
    std::vector<std::vector<Mono>> lam(nf), lam_i(ni);
    for (const Term& t : c->terms) {
        if (!t.implicit) continue;
        auto& dst = is_interm(t.target) ? lam_i[t.target - PSS_MAXF] : lam[t.target];
        dst.insert(dst.end(), t.op.begin(), t.op.end());
    }
    pss_status st = PSS_OK;
    // an intermediate field's equation must be solvable at every mode: psi =
    // rhs / (1 - L_psi(q)) with 1 - L_psi bounded away from zero
    for (int i = 0; i < ni && st == PSS_OK; ++i) {
        for_each_mode(c, [&](const double* q, bool* nyq) {
            if (st != PSS_OK) return;
            double im = 0;
            const double re = op_real_at(lam_i[i], q, nyq, &im);
            const double d = std::hypot(1.0 - re, im), l = std::hypot(re, im);
            if (!(d > 1e-6 * std::max(1.0, l)))
                st = fail(PSS_E_UNSTABLE, "intermediate field '%s': 1 - L(q) = %g vanishes at q = (%g, %g, %g)",
                          c->interms[i].c_str(), d, q[0], q[1], q[2]);
        });
    }
    for (int f = 0; f < nf && st == PSS_OK; ++f) {
        for_each_mode(c, [&](const double* q, bool* nyq) {
            if (st != PSS_OK) return;
            double im = 0;
            const double re = op_real_at(lam[f], q, nyq, &im);
            if (!(1.0 - c->dt * re > 0.0))
                st = fail(PSS_E_UNSTABLE, "field %d: Re(1 - dt L(q)) = %g <= 0 at q = (%g, %g, %g)", f,
                          1.0 - c->dt * re, q[0], q[1], q[2]);
            if (c->fields[f].noisy) {
                double dim = 0;
                const double D = op_real_at(c->fields[f].noise, q, nyq, &dim);
                if (D < 0 || dim != 0)
                    st = fail(PSS_E_INVAL, "field %d: noise operator D(q) = %g is negative", f, D);
            }
        });
    }
    return st;
}

// keep-mask constants of a factor with cutoff num/den of Nyquist
pss::DevMask make_mask(const pss_ctx* c, int rule, int shape, int order) {
    pss::DevMask mk{};
    const int nz = c->ndim == 3 ? c->n[2] : 1;
    const int ns[3] = {c->n[0], c->n[1], nz};
    if (rule == PSS_DEALIAS_NONE) {
        mk.shape = 2;
        mk.ncol = c->n[0] / 2;
        mk.ylo = c->n[1] / 2;
        return mk;
    }
    const int num = 2, den = rule == PSS_DEALIAS_TWO_THIRDS ? 3 : order + 1;
    mk.num = num;
    mk.den = den;
    mk.shape = shape == PSS_SHAPE_PER_AXIS ? 1 : 0;
    int64_t l = 1;
    for (int i = 0; i < 3; ++i) {
        mk.h[i] = ns[i] > 1 ? ns[i] / 2 : 0;
        if (mk.h[i]) l = std::lcm(l, static_cast<int64_t>(mk.h[i]) * mk.h[i]);
    }
    for (int i = 0; i < 3; ++i) mk.w[i] = mk.h[i] ? l / (static_cast<int64_t>(mk.h[i]) * mk.h[i]) : 0;
    mk.den2 = static_cast<int64_t>(den) * den;
    mk.rhs = static_cast<int64_t>(num) * num * l;
    // kept |kx| satisfy den |kx| < num h_x on either shape; the packed column
    // count also keeps column 0 (kx = 0 is always kept)
    int kmax = 0;
    while (den * (kmax + 1) < num * mk.h[0]) ++kmax;
    mk.ncol = std::min(kmax + 1, c->n[0] / 2);
    int ymax = 0;
    while (den * (ymax + 1) < num * mk.h[1]) ++ymax;
    mk.ylo = ymax;
    return mk;
}

pss_status build_plan(pss_ctx* c) {
    using namespace pss;
    DevPlan& P = c->plan;
    P = DevPlan{};
    const int nf = static_cast<int>(c->fields.size());
    P.ndim = c->ndim;
    P.n[0] = c->n[0];
    P.n[1] = c->n[1];
    P.n[2] = c->ndim == 3 ? c->n[2] : 1;
    P.nf = nf;
    for (int i = 0; i < 3; ++i) P.qs[i] = static_cast<float>(2 * M_PI / (P.n[i] * c->dx[i]));
    if (c->ndim <= 2) P.qs[2] = 0.f;
    if (c->ndim == 1) P.qs[1] = 0.f;
    P.dt = static_cast<float>(c->dt);
    const double N = static_cast<double>(c->sites());
    const double dV = c->dx[0] * c->dx[1] * (c->ndim == 3 ? c->dx[2] : 1.0);
    P.inv_n = static_cast<float>(1.0 / N);
    P.amp_pair = static_cast<float>(std::sqrt(c->dt * N / dV));
    P.amp_self = static_cast<float>(std::sqrt(2.0 * c->dt * N / dV));
    P.key0 = static_cast<uint32_t>(c->seed & 0xffffffffu);
    P.key1 = static_cast<uint32_t>(c->seed >> 32);

    // pure (q^2)^j monomials go into the Horner coefficients, the others into
    // the general list
    auto put_mono = [](DevOp& op, const Mono& m) -> int {
        if (m.invq == 0 && m.iq[0] == 0 && m.iq[1] == 0 && m.iq[2] == 0) {
            op.poly[m.q2] += static_cast<float>(m.coef);
            return 0;
        }
        if (op.n >= PSS_MAXM) return -1;
        DevMono& d = op.m[op.n];
        d.coef = static_cast<float>(m.coef);
        d.q2 = static_cast<int8_t>(m.q2);
        d.invq = static_cast<int8_t>(m.invq);
        d.ix = static_cast<int8_t>(m.iq[0]);
        d.iy = static_cast<int8_t>(m.iq[1]);
        d.iz = static_cast<int8_t>(m.iq[2]);
        d.ipow = static_cast<int8_t>((m.iq[0] + m.iq[1] + m.iq[2]) & 3);
        return ++op.n;
    };

    for (size_t id = 0; id < c->ids.size(); ++id)
        if (!is_interm(c->ids[id])) P.fid[c->ids[id]] = static_cast<int32_t>(id);
    const int ni = static_cast<int>(c->interms.size());
    P.ni = ni;
    for (int f = 0; f < nf; ++f) {
        P.noisy[f] = c->fields[f].noisy ? 1 : 0;
        for (const Mono& m : c->fields[f].noise)
            if (put_mono(P.noise_op[f], m) < 0) return fail(PSS_E_UNSUPPORTED, "too many noise monomials");
    }
    // factor slots: fields entering real-space products, with the highest order
    // (indexed by internal code)
    std::vector<int> order(PSS_MAXF + PSS_MAXI, 0);
    for (Term& t : c->terms) {
        if (is_interm(t.target)) {
            // psi = sum_k op_k phi_k / (1 - L_psi): implicit terms build L_psi,
            // explicit ones (one dynamic factor to the first power) op_k
            DevInterm& I = P.interm[t.target - PSS_MAXF];
            t.kind = 4;
            t.slot = t.target - PSS_MAXF;
            if (t.implicit) {
                for (const Mono& m : t.op)
                    if (put_mono(I.den, m) < 0)
                        return fail(PSS_E_UNSUPPORTED, "more than %d implicit monomials on a field", PSS_MAXM);
                continue;
            }
            const int src = t.factors[0].first;
            int k = 0;
            while (k < I.nsrc && I.src[k] != src) ++k;
            if (k == I.nsrc) I.src[I.nsrc++] = src;
            for (const Mono& m : t.op)
                if (put_mono(I.op[k], m) < 0)
                    return fail(PSS_E_UNSUPPORTED, "more than %d monomials on one source of an intermediate field",
                                PSS_MAXM);
            continue;
        }
        if (t.implicit) {
            t.kind = 0;
            t.slot = t.target;
            t.mono0 = P.implicit_op[t.target].n;
            for (const Mono& m : t.op)
                if (put_mono(P.implicit_op[t.target], m) < 0)
                    return fail(PSS_E_UNSUPPORTED, "more than %d implicit monomials on a field", PSS_MAXM);
            continue;
        }
        if (t.factors.size() == 1 && t.factors[0].second == 1) {
            if (P.nd >= PSS_MAXD) return fail(PSS_E_UNSUPPORTED, "more than %d linear explicit terms", PSS_MAXD);
            t.kind = 1;
            t.slot = P.nd;
            t.mono0 = 0;
            DevDirect& d = P.direct[P.nd++];
            d.target = t.target;
            d.src = t.factors[0].first;
            for (const Mono& m : t.op) put_mono(d.op, m);
            continue;
        }
        int ord = 0;
        for (auto& fp : t.factors) ord += fp.second;
        for (auto& fp : t.factors) order[fp.first] = std::max(order[fp.first], ord);
    }
    int gslot[PSS_MAXF + PSS_MAXI];
    P.ng = 0;
    for (int code = 0; code < PSS_MAXF + PSS_MAXI; ++code) {
        gslot[code] = -1;
        if (order[code] > 0) {
            if (P.ng >= PSS_MAXG)
                return fail(PSS_E_UNSUPPORTED, "at most %d distinct fields in real-space products", PSS_MAXG);
            gslot[code] = P.ng;
            P.gfield[P.ng] = code;
            P.mask[P.ng] = make_mask(c, c->rule, c->shape, order[code]);
            ++P.ng;
        }
    }
    // channels; single-monomial terms with the same target and shape share one
    std::vector<DevChannel> chs;
    std::vector<std::tuple<int, int, int, int, int, int>> chan_key;
    for (Term& t : c->terms) {
        if (t.implicit || t.kind == 1 || t.kind == 4) continue;
        const bool single = t.op.size() == 1;
        const auto key = single ? std::make_tuple(t.target, t.op[0].q2, t.op[0].invq, t.op[0].iq[0], t.op[0].iq[1],
                                                  t.op[0].iq[2])
                                : std::make_tuple(-1, 0, 0, 0, 0, 0);
        int ch = -1;
        if (single) {
            for (size_t k = 0; k < chs.size(); ++k)
                if (chan_key[k] == key && chs[k].nprod < PSS_MAXPT) ch = static_cast<int>(k);
        }
        if (ch < 0) {
            ch = static_cast<int>(chs.size());
            chs.push_back(DevChannel{});
            chan_key.push_back(key);
            DevChannel& C = chs.back();
            C.nout = 1;
            C.target[0] = t.target;
            if (single) {
                Mono unit = t.op[0];
                unit.coef = 1.0;
                put_mono(C.op[0], unit);
            } else {
                for (const Mono& m : t.op) put_mono(C.op[0], m);
            }
        }
        DevChannel& C = chs[ch];
        DevProd& pd = C.prod[C.nprod];
        pd.coef = single ? static_cast<float>(t.op[0].coef) : 1.f;
        for (auto& fp : t.factors) pd.pow[gslot[fp.first]] += static_cast<int8_t>(fp.second);
        t.kind = single ? 2 : 3;
        t.slot = ch;
        t.prod = C.nprod;
        t.mono0 = 0;
        ++C.nprod;
    }
    // channels forming the same products (up to one common factor r) for
    // different fields share one transform: the later one becomes another
    // output of the earlier, its operator scaled by r
    {
        auto same_products = [](const DevChannel& x, const DevChannel& y, double* r) {
            if (x.nprod != y.nprod || x.nprod == 0 || x.prod[0].coef == 0.f) return false;
            for (int i = 0; i < x.nprod; ++i) {
                if (std::memcmp(x.prod[i].pow, y.prod[i].pow, sizeof(x.prod[i].pow)) != 0) return false;
                // y_i / x_i == y_0 / x_0, exactly (products of two floats are exact in double)
                if (static_cast<double>(y.prod[i].coef) * x.prod[0].coef !=
                    static_cast<double>(x.prod[i].coef) * y.prod[0].coef)
                    return false;
            }
            *r = static_cast<double>(y.prod[0].coef) / x.prod[0].coef;
            return true;
        };
        auto scaled = [](const DevOp& op, double r) {
            DevOp o = op;
            for (int j = 0; j <= PSS_MAXPOW; ++j) o.poly[j] = static_cast<float>(r * op.poly[j]);
            for (int i = 0; i < op.n; ++i) o.m[i].coef = static_cast<float>(r * op.m[i].coef);
            return o;
        };
        auto has_target = [](const DevChannel& x, int f) {
            for (int o = 0; o < x.nout; ++o)
                if (x.target[o] == f) return true;
            return false;
        };
        std::vector<int> remap(chs.size());
        std::vector<DevChannel> merged;
        for (size_t k = 0; k < chs.size(); ++k) {
            int into = -1;
            double r = 1.0;
            for (size_t j = 0; j < merged.size() && into < 0; ++j)
                if (merged[j].nout < PSS_MAXO && !has_target(merged[j], chs[k].target[0]) &&
                    same_products(merged[j], chs[k], &r))
                    into = static_cast<int>(j);
            if (into >= 0) {
                DevChannel& D = merged[into];
                D.target[D.nout] = chs[k].target[0];
                D.op[D.nout] = r == 1.0 ? chs[k].op[0] : scaled(chs[k].op[0], r);
                ++D.nout;
                remap[k] = into;
            } else {
                remap[k] = static_cast<int>(merged.size());
                merged.push_back(chs[k]);
            }
        }
        if (merged.size() > PSS_MAXCH)
            return fail(PSS_E_UNSUPPORTED, "%zu product channels (at most %d)", merged.size(), PSS_MAXCH);
        P.nch = static_cast<int32_t>(merged.size());
        for (size_t k = 0; k < merged.size(); ++k) P.ch[k] = merged[k];
        for (Term& t : c->terms)
            if (t.kind == 2 || t.kind == 3) t.slot = remap[t.slot];
    }
    // Horner degree of every operator
    auto set_deg = [](DevOp& op) {
        op.deg = 0;
        for (int j = PSS_MAXPOW; j > 0; --j)
            if (op.poly[j] != 0.f) {
                op.deg = j;
                break;
            }
    };
    for (int f = 0; f < nf; ++f) {
        set_deg(P.implicit_op[f]);
        set_deg(P.noise_op[f]);
    }
    for (int d = 0; d < P.nd; ++d) set_deg(P.direct[d].op);
    for (int k = 0; k < P.nch; ++k)
        for (int o = 0; o < P.ch[k].nout; ++o) set_deg(P.ch[k].op[o]);
    for (int i = 0; i < ni; ++i) {
        set_deg(P.interm[i].den);
        for (int k = 0; k < P.interm[i].nsrc; ++k) set_deg(P.interm[i].op[k]);
    }
    // kernels without the general-monomial code unless some operator needs it
    P.general = 0;
    for (int f = 0; f < nf; ++f) P.general |= (P.implicit_op[f].n > 0) | (P.noise_op[f].n > 0);
    for (int d = 0; d < P.nd; ++d) P.general |= P.direct[d].op.n > 0;
    for (int k = 0; k < P.nch; ++k)
        for (int o = 0; o < P.ch[k].nout; ++o) P.general |= P.ch[k].op[o].n > 0;
    P.general |= ni > 0;  // intermediates are evaluated by the general-operator code
    for (int f = 0; f < nf; ++f) {  // boundary frames already on the device
        P.frame[f] = c->d_frame[f];
        P.nframe[f] = c->d_frame[f] && f < static_cast<int>(c->frames.size())
                          ? static_cast<int32_t>(c->frames[f].size()) : 0;
    }
    return PSS_OK;
}

int pick_pow2(int want, int lo, int hi) {
    int v = 1;
    while (v < want) v <<= 1;
    return std::max(lo, std::min(hi, v));
}

// Launch geometry.  Defaults come from the sizes; pss_tuning_set can force any
// of tc, to, tz, rb (powers of two) and pu, px, py (points per thread: 4, 8 or
// 16) before the plan is built; on mixed-radix lattices tc and py are lines
// per column / y-pass block.
pss_status choose_geometry(pss_ctx* c) {
    const int nf = static_cast<int>(c->fields.size());
    const int ng = std::max(1, c->plan.ng);
    const int nx = c->n[0], ny = c->n[1];
    const int nz = c->ndim == 3 ? c->n[2] : 1;
    const int ncols = nx / 2;
    pss::Geo& g = c->geo;
    g = pss::Geo{};
    g.nz = nz;
    if (c->ndim == 1) {
        // one block holds the line, 4 points per thread (no tunable geometry)
        c->lu = nx;
        g.tc = 1;
        g.to = 1;
        g.pu = g.px = 4;
        g.ntile = 1;
        g.nublk = 1;
        g.nrowblk = 1;
        g.rb = 2;
        if (is_pow2(nx)) {
            if (pss::line1d_lds_bytes(nx) > 160 * 1024)
                return fail(PSS_E_UNSUPPORTED, "line needs more LDS than a workgroup has");
        } else {
            // mixed-radix lines keep their spectra in LDS
            const int NF = nf <= 1 ? 1 : (nf == 2 ? 2 : 4);
            const size_t lds = pss::line1d_mr_lds_bytes(nx, NF, c->plan.ng);
            if (lds > 160 * 1024)
                return fail(PSS_E_UNSUPPORTED,
                            "a line of %d sites with %d fields and %d factor fields needs %zu bytes of LDS "
                            "(160 KiB at most)", nx, nf, c->plan.ng, lds);
        }
        return PSS_OK;
    }
    if (c->mixed) {
        // spectra in LDS, one block per x row; the column launch (and the 3D
        // y pass) takes tc lines of neighbouring kx per block.  One line per
        // block is the default: the blocks are XCD-ordered, so neighbouring
        // columns share their cache lines in one L2, and the smaller LDS
        // footprint keeps more blocks per CU (960^2 Model B: 54.2, 56.7 and
        // 73.5 us per step at tc = 1, 2, 4)
        c->lu = c->ndim == 3 ? nz : ny;
        const int NF = nf <= 1 ? 1 : (nf == 2 ? 2 : 4);
        auto fits1 = [&](auto bytes) { return bytes(1) <= 160 * 1024 ? 1 : 0; };
        g.tc = fits1([&](int tc) { return pss::mr2_col_lds_bytes(c->lu, NF, tc); });
        g.py = c->ndim == 3 ? fits1([&](int tc) { return pss::mr3_ypass_lds_bytes(ny, tc); }) : 1;
        // pss_tuning_set may force either (a divisor of Nx that fits)
        auto forced = [&](const char* key, int& v, auto bytes) {
            auto it = c->tune.find(key);
            if (it == c->tune.end()) return true;
            const int64_t w = it->second;
            if (w < 1 || w > 64 || nx % w != 0 || bytes(static_cast<int>(w)) > 160 * 1024) return false;
            v = static_cast<int>(w);
            return true;
        };
        if (!forced("tc", g.tc, [&](int tc) { return pss::mr2_col_lds_bytes(c->lu, NF, tc); }) ||
            (c->ndim == 3 && !forced("py", g.py, [&](int tc) { return pss::mr3_ypass_lds_bytes(ny, tc); })))
            return fail(PSS_E_UNSUPPORTED, "forced tc / py must divide Nx and fit the LDS");
        g.to = 1;
        g.pu = g.px = 4;
        g.ntile = ncols;
        g.nublk = (nx / std::max(g.tc, 1)) * (c->ndim == 3 ? ny : 1);
        g.nrowblk = ny * nz;
        g.rb = 2;
        const size_t lr = pss::mr2_row_lds_bytes(nx, c->plan.ng);
        if (g.tc == 0 || g.py == 0 || lr > 160 * 1024)
            return fail(PSS_E_UNSUPPORTED, "lattice needs more LDS than a workgroup has (%zu, %zu bytes)",
                        pss::mr2_col_lds_bytes(c->lu, NF, 1), lr);
        return PSS_OK;
    }
    auto tuned = [&](const char* key, int def) {
        auto it = c->tune.find(key);
        return it == c->tune.end() ? def : static_cast<int>(it->second);
    };
    auto pow2 = [](int v) { return v > 0 && (v & (v - 1)) == 0; };
    c->lu = c->ndim == 2 ? ny : nz;
    const int lu = c->lu;
    // default: the fewest points per thread (most threads per line) that keep
    // a line within one 256-thread block; fewer points per thread measured
    // faster for every kernel (lower register use, more waves in flight)
    auto few_points = [](int L, int cap) { return std::min(cap, std::max(std::min(4, L), L / 256)); };
    g.pu = tuned("pu", few_points(lu, pss::max_points(lu, pss::field_slots(nf))));
    g.px = tuned("px", few_points(nx, pss::max_points(nx, pss::field_slots(ng))));
    if (!pow2(g.pu) || g.pu > pss::max_points(lu, pss::field_slots(nf)) || !pow2(g.px) ||
        g.px > pss::max_points(nx, pss::field_slots(ng)))
        return fail(PSS_E_UNSUPPORTED, "points per thread must be a power of two up to the variant limit");
    const int tu = lu / g.pu;
    if (c->ndim == 2) {
        g.tc = tuned("tc", std::min(std::max(1, 256 / tu), ncols));
        g.to = 1;
    } else {
        g.tc = tuned("tc", std::min(4, ncols));
        g.to = tuned("to", std::max(1, std::min(256 / (g.tc * tu), ny / 2)));
    }
    if (!pow2(g.tc) || g.tc > ncols || !pow2(g.to) || g.to > std::max(1, ny / 2))
        return fail(PSS_E_UNSUPPORTED, "tile width tc must be a power of two up to Nx/2, to up to Ny/2");
    if (g.tc * g.to * tu > 256)
        return fail(PSS_E_UNSUPPORTED, "update kernel block of %d threads exceeds 256", g.tc * g.to * tu);
    g.ntile = ncols / g.tc;
    g.nublk = c->ndim == 2 ? g.ntile : g.ntile * (ny / g.to);
    if (c->ndim == 3) {
        // y pass: TC lines of Ny points per z share a block of <= 256 threads
        g.py = tuned("py", std::min(pss::max_points(ny, 1),
                                    std::max(few_points(ny, pss::max_points(ny, 1)), pick_pow2(g.tc * ny / 256, 1, 16))));
        if (!pow2(g.py) || g.py > pss::max_points(ny, 1))
            return fail(PSS_E_UNSUPPORTED, "points per thread must be a power of two up to the variant limit");
        const int ty = g.tc * (ny / g.py);
        if (ty > 256) return fail(PSS_E_UNSUPPORTED, "y line length %d needs more than 256 threads", ny);
        g.tz = tuned("tz", std::max(1, std::min(256 / ty, nz)));
        if (!pow2(g.tz) || g.tz > nz || g.tz * ty > 256)
            return fail(PSS_E_UNSUPPORTED, "y-pass block (tz = %d) is too large", g.tz);
        g.nyblk = g.ntile * (nz / g.tz);
        if (pss::ypass_lds_bytes(ny, g.py, g.tc, g.tz) > 160 * 1024)
            return fail(PSS_E_UNSUPPORTED, "y pass needs more LDS than a workgroup has");
    }
    // x kernel: RB rows (pairs of T threads); aim for >= 512 blocks, 64..256 threads
    const int tx = nx / g.px;
    if (tx > 256) return fail(PSS_E_UNSUPPORTED, "row length %d needs more than 256 threads", nx);
    const int rows = ny * nz;
    const int rb_lo = std::max(2, 2 * (64 / tx));
    const int rb_hi = std::max(2, 2 * (256 / tx));
    int rb = pick_pow2(std::max(2, rows / 512), rb_lo, rb_hi);
    rb = tuned("rb", std::min(rb, ny));  // a block's rows share z
    if (!pow2(rb) || rb < 2 || rb > ny || (rb / 2) * tx > 256)
        return fail(PSS_E_UNSUPPORTED, "x-kernel block of %d rows is not valid", rb);
    g.rb = rb;
    g.nrowblk = rows / rb;
    g.tc_log2 = 0;
    while ((1 << g.tc_log2) < g.tc) ++g.tc_log2;
    g.rb_log2 = 0;
    while ((1 << g.rb_log2) < g.rb) ++g.rb_log2;
    const size_t lu_lds = pss::update_lds_bytes(lu, g.pu, g.tc, g.to);
    const size_t lx_lds = pss::xrow_lds_bytes(nx, g.px, rb);
    if (lu_lds > 160 * 1024 || lx_lds > 160 * 1024)
        return fail(PSS_E_UNSUPPORTED, "lattice needs more LDS than a workgroup has (%zu, %zu bytes)", lu_lds,
                    lx_lds);
    return PSS_OK;
}

void free_device(pss_ctx* c) {
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
    auto rel = [](auto*& p) {
        if (p) (void)hipFree(p);
        p = nullptr;
    };
    for (size_t f = 0; f < c->d_state.size(); ++f) {
        if (f < PSS_MAXF && c->d_state[f] == c->bound[f])
            c->d_state[f] = nullptr;  // the caller's memory: not ours to free
        else
            rel(c->d_state[f]);
    }
    for (size_t k = 0; k < c->d_chan_x.size(); ++k)
        if (c->d_chan_x[k] != c->d_chan[k]) rel(c->d_chan_x[k]);
    c->d_chan_x.clear();
    for (auto*& p : c->d_chan) rel(p);
    for (auto*& p : c->d_v) rel(p);
    rel(c->d_plan);
    rel(c->d_step);
    rel(c->d_tw_u);
    rel(c->d_tw_x);
    rel(c->d_tw_y);
    rel(c->d_tmp);
    rel(c->d_tmp2);
    rel(c->d_real);
    rel(c->d_shell_acc);
    rel(c->d_member_u);
    rel(c->d_member_x);
    for (auto*& p : c->d_frame) rel(p);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    c->stream = nullptr;
    c->own_stream = false;
    c->planned = false;
}

uint32_t* flag_of(pss_ctx* c) { return c->d_step ? reinterpret_cast<uint32_t*>(c->d_step + 1) : nullptr; }

// Debug mode only: wait for the kernel just enqueued and report, by kernel
// and step, a launch or execution error or the first non-finite state value.
pss_status debug_check(pss_ctx* c, const char* kernel, int64_t step) {
    if (!c->debug_sync) return PSS_OK;
    const hipError_t e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess)
        return fail(PSS_E_HIP, "%s (step %lld): %s", kernel, static_cast<long long>(step), hipGetErrorString(e));
    uint32_t f = 0;
    HIP_TRY(hipMemcpy(&f, flag_of(c), sizeof(f), hipMemcpyDeviceToHost));
    if (!f) return PSS_OK;
    const uint32_t zero = 0;
    HIP_TRY(hipMemcpy(flag_of(c), &zero, sizeof(zero), hipMemcpyHostToDevice));
    return fail(PSS_E_NONFINITE, "a non-finite value appeared in the state (field mask 0x%x) in %s of step %lld", f,
                kernel, static_cast<long long>(step));
}

pss::LaunchArgs args(pss_ctx* c, int step_off = 0) {
    pss::LaunchArgs a{};
    a.stream = c->stream;
    a.plan = c->d_plan;
    for (size_t f = 0; f < c->d_state.size(); ++f) a.bufs.S[f] = c->d_state[f];
    for (size_t k = 0; k < c->d_chan.size(); ++k) a.bufs.N[k] = c->d_chan[k];
    for (size_t g = 0; g < c->d_v.size(); ++g) a.bufs.V[g] = c->d_v[g];
    a.geo = c->geo;
    a.step_ctr = c->d_step;
    a.flag = flag_of(c);
    a.members = c->d_member_u;
    a.plans = c->d_plan;
    a.nmem = 1;
    a.general = c->plan.general != 0;
    a.step_off = step_off;
    a.tw_u = c->d_tw_u;
    a.tw_x = c->d_tw_x;
    a.tw_y = c->d_tw_y;
    a.dim = c->ndim;
    a.ng = c->plan.ng;
    a.nx = c->n[0];
    a.ny = c->n[1];
    a.nz = c->n[2];
    return a;
}

// x-kernel arguments: channel outputs go to the y-pass layout in 3D
pss::LaunchArgs xargs(pss_ctx* c) {
    pss::LaunchArgs a = args(c);
    for (size_t k = 0; k < c->d_chan_x.size(); ++k) a.bufs.N[k] = c->d_chan_x[k];
    a.members = c->d_member_x;
    return a;
}

// member-table entries of the update kernel and the x kernel of a context
pss::Member member_u(pss_ctx* c) {
    const pss::LaunchArgs a = args(c);
    return pss::Member{a.bufs, c->d_step, flag_of(c)};
}
pss::Member member_x(pss_ctx* c) {
    const pss::LaunchArgs a = xargs(c);
    return pss::Member{a.bufs, c->d_step, flag_of(c)};
}

hipError_t y_inverse_factors(pss_ctx* c) {
    pss::YArgs ya{};
    ya.n = c->plan.ng;
    for (int g = 0; g < ya.n; ++g) {
        ya.src[g] = c->d_v[g];
        ya.dst[g] = c->d_v[g];  // in place: each line is read whole before it is written
        ya.ncol[g] = c->plan.mask[g].ncol;
    }
    return pss::launch_ypass(pss::MODE_YINV, c->n[1], ya, args(c));
}

hipError_t y_forward_channels(pss_ctx* c) {
    pss::YArgs ya{};
    ya.n = c->plan.nch;
    for (int k = 0; k < ya.n; ++k) {
        ya.src[k] = c->d_chan_x[k];
        ya.dst[k] = c->d_chan[k];
        ya.ncol[k] = c->n[0] / 2;
    }
    return pss::launch_ypass(pss::MODE_YFWD, c->n[1], ya, args(c));
}

// 3D mixed-radix lattices: y transforms (sign -1 forward, +1 inverse) of n
// arrays in place
hipError_t mr_ypass(pss_ctx* c, int sign, float2* const* arrs, int n) {
    pss::YArgs ya{};
    ya.n = n;
    for (int i = 0; i < n; ++i) {
        ya.src[i] = arrs[i];
        ya.dst[i] = arrs[i];
    }
    return pss::launch_mr3_ypass(sign, ya, args(c));
}

bool has_frames(const pss_ctx* c) {
    for (const auto& fr : c->frames)
        if (!fr.empty()) return true;
    return false;
}

// copy every field's frame to the device and point the plan at it (the
// caller uploads the plan)
pss_status upload_frames(pss_ctx* c) {
    for (int f = 0; f < PSS_MAXF; ++f) {
        if (c->d_frame[f]) (void)hipFree(c->d_frame[f]);
        c->d_frame[f] = nullptr;
        c->plan.frame[f] = nullptr;
        c->plan.nframe[f] = 0;
        if (f >= static_cast<int>(c->frames.size()) || c->frames[f].empty()) continue;
        const auto& fr = c->frames[f];
        HIP_TRY(hipMalloc(&c->d_frame[f], sizeof(int2) * fr.size()));
        HIP_TRY(hipMemcpy(c->d_frame[f], fr.data(), sizeof(int2) * fr.size(), hipMemcpyHostToDevice));
        c->plan.frame[f] = c->d_frame[f];
        c->plan.nframe[f] = static_cast<int32_t>(fr.size());
    }
    return PSS_OK;
}

pss_status upload_plan(pss_ctx* c) {
    HIP_TRY(hipStreamSynchronize(c->stream));
    HIP_TRY(hipMemcpy(c->d_plan, &c->plan, sizeof(pss::DevPlan), hipMemcpyHostToDevice));
    ++c->plan_gen;
    return PSS_OK;
}

pss_status materialize(pss_ctx* c) {
    if (c->planned) return PSS_OK;
    pss_status st = validate(c);
    if (st) return st;
    if ((st = build_plan(c))) return st;
    if ((st = choose_geometry(c))) return st;
    if (!c->stream) {
        HIP_TRY(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        c->own_stream = true;
    }
    const size_t bytes = sizeof(float2) * static_cast<size_t>(c->packed());
    const int nf = static_cast<int>(c->fields.size());
    c->d_state.assign(nf, nullptr);
    c->d_chan.assign(c->plan.nch, nullptr);
    c->d_v.assign(c->plan.ng, nullptr);
    for (int f = 0; f < nf; ++f) {
        float2*& p = c->d_state[f];
        if (c->bound[f]) {
            // caller-owned memory (pss_field_bind): it must be device memory
            hipPointerAttribute_t at{};
            HIP_TRY(hipPointerGetAttributes(&at, c->bound[f]));
            if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged)
                return fail(PSS_E_INVAL, "the memory bound to field %d is not device memory", f);
            p = static_cast<float2*>(c->bound[f]);
        } else {
            HIP_TRY(hipMalloc(&p, bytes));
        }
        HIP_TRY(hipMemset(p, 0, bytes));
    }
    // workspaces: zeros, or all-ones bytes (a NaN in every float) in debug
    // mode, so that a read before the first write reaches the state as NaN
    const int fill = c->debug_sync ? 0xFF : 0;
    for (auto*& p : c->d_chan) {
        HIP_TRY(hipMalloc(&p, bytes));
        HIP_TRY(hipMemset(p, fill, bytes));
    }
    c->d_chan_x = c->d_chan;
    if (c->ndim == 3 && !c->mixed) {
        for (auto*& p : c->d_chan_x) {
            HIP_TRY(hipMalloc(&p, bytes));
            HIP_TRY(hipMemset(p, fill, bytes));
        }
    }
    for (auto*& p : c->d_v) {
        HIP_TRY(hipMalloc(&p, bytes));
        HIP_TRY(hipMemset(p, fill, bytes));
    }
    HIP_TRY(hipMalloc(&c->d_tmp, bytes));
    HIP_TRY(hipMalloc(&c->d_tmp2, bytes));
    HIP_TRY(hipMalloc(&c->d_real, sizeof(float) * static_cast<size_t>(c->sites())));
    if (c->debug_sync) {
        HIP_TRY(hipMemset(c->d_tmp, fill, bytes));
        HIP_TRY(hipMemset(c->d_tmp2, fill, bytes));
        HIP_TRY(hipMemset(c->d_real, fill, sizeof(float) * static_cast<size_t>(c->sites())));
    }
    HIP_TRY(hipMalloc(&c->d_plan, sizeof(pss::DevPlan)));
    // the step counter and, in the next word, the non-finite flag
    HIP_TRY(hipMalloc(&c->d_step, 2 * sizeof(uint64_t)));
    HIP_TRY(hipMemset(c->d_step, 0, 2 * sizeof(uint64_t)));
    const auto twx = twiddles(c->n[0]);
    const auto twu = twiddles(c->lu);
    HIP_TRY(hipMalloc(&c->d_tw_x, sizeof(float2) * twx.size()));
    HIP_TRY(hipMalloc(&c->d_tw_u, sizeof(float2) * twu.size()));
    HIP_TRY(hipMemcpy(c->d_tw_x, twx.data(), sizeof(float2) * twx.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->d_tw_u, twu.data(), sizeof(float2) * twu.size(), hipMemcpyHostToDevice));
    const auto twy = twiddles(c->n[1]);
    HIP_TRY(hipMalloc(&c->d_tw_y, sizeof(float2) * twy.size()));
    HIP_TRY(hipMemcpy(c->d_tw_y, twy.data(), sizeof(float2) * twy.size(), hipMemcpyHostToDevice));
    if (pss_status s = upload_frames(c)) return s;
    HIP_TRY(hipMemcpy(c->d_plan, &c->plan, sizeof(pss::DevPlan), hipMemcpyHostToDevice));
    if (c->ndim == 1) HIP_TRY(pss::line1d_setup(c->n[0]));
    if (c->mixed) HIP_TRY(pss::mr2_setup());
    HIP_TRY(hipMalloc(&c->d_member_u, sizeof(pss::Member)));
    HIP_TRY(hipMalloc(&c->d_member_x, sizeof(pss::Member)));
    const pss::Member mu = member_u(c), mx = member_x(c);
    HIP_TRY(hipMemcpy(c->d_member_u, &mu, sizeof(mu), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->d_member_x, &mx, sizeof(mx), hipMemcpyHostToDevice));
    HIP_TRY(hipDeviceSynchronize());
    c->planned = true;
    c->dirty = true;
    c->steps_taken = 0;
    return PSS_OK;
}

// Rebuild the channel arrays from the current state (masked inverse along the
// update axis, then the real-space products).
pss_status prologue(pss_ctx* c) {
    const int nf = static_cast<int>(c->fields.size());
    if (c->ndim == 1) {  // a 1D launch forms its first step's products from the state itself
        c->dirty = false;
        return PSS_OK;
    }
    pss::LaunchArgs a = args(c);
    if (c->mixed) {
        HIP_TRY(pss::launch_mr2_col(pss::MODE_PROLOGUE, nf, a));
        if (c->plan.nch > 0) {
            if (c->ndim == 3) HIP_TRY(mr_ypass(c, 1, c->d_v.data(), c->plan.ng));
            HIP_TRY(pss::launch_mr2_row(pss::MODE_STEP, a));
            if (c->ndim == 3) HIP_TRY(mr_ypass(c, -1, c->d_chan.data(), c->plan.nch));
        }
        c->dirty = false;
        return PSS_OK;
    }
    HIP_TRY(pss::launch_update(pss::MODE_PROLOGUE, c->lu, nf, a));
    if (c->plan.nch > 0) {
        if (c->ndim == 3) HIP_TRY(y_inverse_factors(c));
        HIP_TRY(pss::launch_xrow(pss::MODE_STEP, c->n[0], c->plan.ng, xargs(c)));
        if (c->ndim == 3) HIP_TRY(y_forward_channels(c));
    }
    c->dirty = false;
    return PSS_OK;
}

// Report (and clear) the non-finite flag that the update kernel raises when
// a new state value is NaN or infinite.  The caller has synchronised.
pss_status take_nonfinite(pss_ctx* c) {
    if (!c->planned) return PSS_OK;
    uint32_t f = 0;
    HIP_TRY(hipMemcpy(&f, flag_of(c), sizeof(f), hipMemcpyDeviceToHost));
    if (!f) return PSS_OK;
    const uint32_t zero = 0;
    HIP_TRY(hipMemcpy(flag_of(c), &zero, sizeof(zero), hipMemcpyHostToDevice));
    return fail(PSS_E_NONFINITE, "a non-finite value appeared in the state (field mask 0x%x) at or before step %lld",
                f, static_cast<long long>(c->steps_taken));
}

// Before the context enqueues work on its own stream: wait for the last batch
// step that touched it, and note that its stream has new work (a batch then
// orders itself after it).  Batches order themselves lazily, so that a batch
// step costs no per-member API calls while the members are left alone.
pss_status begin_work(pss_ctx* c) {
    if (c->after_batch) {
        HIP_TRY(hipStreamWaitEvent(c->stream, c->after_batch, 0));
        c->after_batch = nullptr;
    }
    ++c->enq_gen;
    return PSS_OK;
}

// Order the batch stream after the members' own work and after other batches
// holding them; rebuild stale channel arrays first.
pss_status batch_order_before(pss_batch* b, const std::vector<int>& which) {
    for (int i : which) {
        pss_ctx* c = b->mem[i];
        if (c->dirty) {
            if (pss_status s = begin_work(c)) return s;
            if (pss_status s = prologue(c)) return s;
        }
        if (c->stream == b->stream) continue;
        if (c->after_batch && c->after_batch != b->ev) HIP_TRY(hipStreamWaitEvent(b->stream, c->after_batch, 0));
        if (c->enq_gen != b->seen[i]) {
            HIP_TRY(hipEventRecord(b->ev, c->stream));
            HIP_TRY(hipStreamWaitEvent(b->stream, b->ev, 0));
            b->seen[i] = c->enq_gen;
        }
    }
    return PSS_OK;
}

// after batch work: the members' own later work waits for it
pss_status batch_order_after(pss_batch* b, const std::vector<int>& which) {
    HIP_TRY(hipEventRecord(b->ev, b->stream));
    for (int i : which) {
        pss_ctx* c = b->mem[i];
        if (c->stream != b->stream) c->after_batch = b->ev;
    }
    return PSS_OK;
}

// clear the flag when the state is replaced (uploads, loads)
pss_status clear_nonfinite(pss_ctx* c) {
    const uint32_t zero = 0;
    HIP_TRY(hipMemcpy(flag_of(c), &zero, sizeof(zero), hipMemcpyHostToDevice));
    return PSS_OK;
}

pss_status state_to_real(pss_ctx* c, int field);
pss_status forward_to_state(pss_ctx* c, int field);

pss_status enqueue_steps(pss_ctx* c, int64_t k) {
    const int nf = static_cast<int>(c->fields.size());
    if (c->ndim == 1) {  // one launch takes the whole chunk and moves the counter on
        pss::LaunchArgs a = args(c);
        a.nsteps = static_cast<int>(k);
        a.advance = 1;
        HIP_TRY(pss::launch_line1d(pss::MODE_STEP, c->n[0], nf, a));
        return debug_check(c, "line1d_kernel", c->steps_taken);
    }
    // A framed lattice rebuilds every step's factors and products from the
    // framed state (the prologue after the frames), so its steps run only the
    // update launch: the product launches of the unframed state would be
    // overwritten unread.
    const bool framed = has_frames(c);
    // in 2D the last x kernel of the sequence moves the step counter on
    const bool x_advances = c->ndim == 2 && c->plan.nch > 0 && !framed;
    for (int64_t i = 0; i < k; ++i) {
        pss::LaunchArgs a = args(c, static_cast<int>(i));
        const int64_t at = c->steps_taken + i;
#define PSS_CHECKED(launch, name)                                 \
    do {                                                          \
        HIP_TRY(launch);                                          \
        if (pss_status s_ = debug_check(c, name, at)) return s_;  \
    } while (0)
        if (c->mixed) {
            PSS_CHECKED(pss::launch_mr2_col(pss::MODE_STEP, nf, a), "mr2_col_kernel");
            if (c->plan.nch > 0 && !framed) {
                if (c->ndim == 3) PSS_CHECKED(mr_ypass(c, 1, c->d_v.data(), c->plan.ng), "mr3_ypass_kernel(inverse)");
                a.advance = (x_advances && i == k - 1) ? k : 0;
                PSS_CHECKED(pss::launch_mr2_row(pss::MODE_STEP, a), "mr2_row_kernel");
                if (c->ndim == 3)
                    PSS_CHECKED(mr_ypass(c, -1, c->d_chan.data(), c->plan.nch), "mr3_ypass_kernel(forward)");
            }
        } else {
            PSS_CHECKED(pss::launch_update(pss::MODE_STEP, c->lu, nf, a), "update_kernel");
            if (c->plan.nch > 0 && !framed) {
                if (c->ndim == 3) PSS_CHECKED(y_inverse_factors(c), "ypass_kernel(inverse)");
                pss::LaunchArgs ax = xargs(c);
                ax.advance = (x_advances && i == k - 1) ? k : 0;
                PSS_CHECKED(pss::launch_xrow(pss::MODE_STEP, c->n[0], c->plan.ng, ax), "xrow_kernel");
                if (c->ndim == 3) PSS_CHECKED(y_forward_channels(c), "ypass_kernel(forward)");
            }
        }
#undef PSS_CHECKED
        if (framed) {
            // boundary frames: each framed field through real space, then the
            // factors and channels of the next step from the framed state
            for (int f = 0; f < nf; ++f) {
                if (f >= static_cast<int>(c->frames.size()) || c->frames[f].empty()) continue;
                if (pss_status s = state_to_real(c, f)) return s;
                HIP_TRY(pss::launch_apply_frame(c->stream, c->d_real, c->d_frame[f],
                                                static_cast<int>(c->frames[f].size())));
                if (pss_status s = forward_to_state(c, f)) return s;
            }
            if (pss_status s = prologue(c)) return s;
            if (pss_status s = debug_check(c, "frames and products", at)) return s;
        }
    }
    if (!x_advances) HIP_TRY(pss::launch_advance(c->stream, c->d_step, k));
    return PSS_OK;
}

// real-space array on the device (d_real) -> Fourier state of `field`
pss_status forward_to_state(pss_ctx* c, int field) {
    pss::LaunchArgs a = args(c);
    if (c->ndim == 1) {
        a.bufs.real_in = c->d_real;
        a.bufs.sel = field;
        HIP_TRY(pss::launch_line1d(pss::MODE_FWD_STORE, c->n[0], 1, a));
        return PSS_OK;
    }
    if (c->mixed) {
        a.bufs.real_in = c->d_real;
        a.bufs.out = c->d_tmp;
        HIP_TRY(pss::launch_mr2_row(pss::MODE_R2C_IN, a));
        if (c->ndim == 3) HIP_TRY(mr_ypass(c, -1, &c->d_tmp, 1));
        a.bufs.in = c->d_tmp;
        a.bufs.sel = field;
        HIP_TRY(pss::launch_mr2_col(pss::MODE_FWD_STORE, 1, a));
        return PSS_OK;
    }
    a.bufs.real_in = c->d_real;
    a.bufs.out = c->d_tmp;
    HIP_TRY(pss::launch_xrow(pss::MODE_R2C_IN, c->n[0], 1, a));
    const float2* in = c->d_tmp;
    if (c->ndim == 3) {
        pss::YArgs ya{};
        ya.n = 1;
        ya.src[0] = c->d_tmp;
        ya.dst[0] = c->d_tmp2;
        ya.ncol[0] = c->n[0] / 2;
        HIP_TRY(pss::launch_ypass(pss::MODE_YFWD, c->n[1], ya, a));
        in = c->d_tmp2;
    }
    a.bufs.in = in;
    a.bufs.sel = field;
    HIP_TRY(pss::launch_update(pss::MODE_FWD_STORE, c->lu, 1, a));
    return PSS_OK;
}

// Fourier state of `field` -> real-space array on the device (d_real)
pss_status state_to_real(pss_ctx* c, int field) {
    pss::LaunchArgs a = args(c);
    if (c->ndim == 1) {
        a.bufs.sel = field;
        a.bufs.real_out = c->d_real;
        HIP_TRY(pss::launch_line1d(pss::MODE_INV_OUT, c->n[0], 1, a));
        return PSS_OK;
    }
    if (c->mixed) {
        a.bufs.sel = field;
        a.bufs.out = c->d_tmp;
        HIP_TRY(pss::launch_mr2_col(pss::MODE_INV_OUT, 1, a));
        if (c->ndim == 3) HIP_TRY(mr_ypass(c, 1, &c->d_tmp, 1));
        a.bufs.in = c->d_tmp;
        a.bufs.real_out = c->d_real;
        HIP_TRY(pss::launch_mr2_row(pss::MODE_C2R_OUT, a));
        return PSS_OK;
    }
    a.bufs.sel = field;
    a.bufs.out = c->d_tmp;
    HIP_TRY(pss::launch_update(pss::MODE_INV_OUT, c->lu, 1, a));
    if (c->ndim == 3) {
        pss::YArgs ya{};
        ya.n = 1;
        ya.src[0] = c->d_tmp;
        ya.dst[0] = c->d_tmp;
        ya.ncol[0] = c->n[0] / 2;
        HIP_TRY(pss::launch_ypass(pss::MODE_YINV, c->n[1], ya, a));
    }
    a.bufs.in = c->d_tmp;
    a.bufs.real_out = c->d_real;
    HIP_TRY(pss::launch_xrow(pss::MODE_C2R_OUT, c->n[0], 1, a));
    return PSS_OK;
}

// intermediate field i, computed from the current state -> real-space array
// on the device (d_real)
pss_status interm_to_real(pss_ctx* c, int i) {
    pss::LaunchArgs a = args(c);
    if (c->ndim == 1) {
        a.bufs.sel = i;
        a.bufs.real_out = c->d_real;
        HIP_TRY(pss::launch_line1d(pss::MODE_INTERM_OUT, c->n[0], static_cast<int>(c->fields.size()), a));
        return PSS_OK;
    }
    if (c->mixed) {
        a.bufs.sel = i;
        a.bufs.out = c->d_tmp;
        HIP_TRY(pss::launch_mr2_col(pss::MODE_INTERM_OUT, static_cast<int>(c->fields.size()), a));
        if (c->ndim == 3) HIP_TRY(mr_ypass(c, 1, &c->d_tmp, 1));
        a.bufs.in = c->d_tmp;
        a.bufs.real_out = c->d_real;
        HIP_TRY(pss::launch_mr2_row(pss::MODE_C2R_OUT, a));
        return PSS_OK;
    }
    a.bufs.sel = i;
    a.bufs.out = c->d_tmp;
    HIP_TRY(pss::launch_update(pss::MODE_INTERM_OUT, c->lu, static_cast<int>(c->fields.size()), a));
    if (c->ndim == 3) {
        pss::YArgs ya{};
        ya.n = 1;
        ya.src[0] = c->d_tmp;
        ya.dst[0] = c->d_tmp;
        ya.ncol[0] = c->n[0] / 2;
        HIP_TRY(pss::launch_ypass(pss::MODE_YINV, c->n[1], ya, a));
    }
    a.bufs.in = c->d_tmp;
    a.bufs.real_out = c->d_real;
    HIP_TRY(pss::launch_xrow(pss::MODE_C2R_OUT, c->n[0], 1, a));
    return PSS_OK;
}

pss_status graph_for(pss_ctx* c, int64_t k, hipGraphExec_t* out) {
    auto it = c->graphs.find(k);
    if (it != c->graphs.end()) {
        *out = it->second;
        return PSS_OK;
    }
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    pss_status st = enqueue_steps(c, k);
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    HIP_TRY(e);
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIP_TRY(e);
    c->graphs[k] = ex;
    *out = ex;
    return PSS_OK;
}

constexpr int64_t kGraphSteps = 50;

bool same_class(const pss_ctx* a, const pss_ctx* b) {
    return a->n[0] == b->n[0] && a->n[1] == b->n[1] && a->fields.size() == b->fields.size() &&
           a->interms.size() == b->interms.size() &&
           a->plan.ng == b->plan.ng && a->plan.nch == b->plan.nch && a->plan.general == b->plan.general &&
           std::memcmp(&a->geo, &b->geo, sizeof(pss::Geo)) == 0;
}

void free_batch(pss_batch* b) {
    for (auto& kv : b->graphs) (void)hipGraphExecDestroy(kv.second);
    b->graphs.clear();
    for (auto& cl : b->cls) {
        if (cl.d_u) (void)hipFree(cl.d_u);
        if (cl.d_x) (void)hipFree(cl.d_x);
        if (cl.d_plans) (void)hipFree(cl.d_plans);
        cl.d_u = cl.d_x = nullptr;
        cl.d_plans = nullptr;
    }
    if (b->d_ctrs) (void)hipFree(b->d_ctrs);
    b->d_ctrs = nullptr;
    if (b->d_flags) (void)hipFree(b->d_flags);
    b->d_flags = nullptr;
    if (b->ev) (void)hipEventDestroy(b->ev);
    b->ev = nullptr;
}

// copy the plans of members whose coefficients changed since the last step
pss_status batch_refresh_plans(pss_batch* b) {
    for (auto& cl : b->cls)
        for (size_t j = 0; j < cl.idx.size(); ++j) {
            pss_ctx* m = b->mem[cl.idx[j]];
            if (cl.gen[j] == m->plan_gen) continue;
            HIP_TRY(hipMemcpyAsync(cl.d_plans + j, m->d_plan, sizeof(pss::DevPlan), hipMemcpyDeviceToDevice,
                                   b->stream));
            cl.gen[j] = m->plan_gen;
        }
    return PSS_OK;
}

// Work lists of the fused launches: every class whose lattices fit the fused
// kernels (one field, operators without general monomials, 4 points per
// thread, 256-thread update blocks, lines of 64 .. 1024).  The fused x launch
// takes 256-thread blocks of 2048/Nx rows: rows per block only regroup the
// same per-row arithmetic.
void batch_plan_fused(pss_batch* b) {
    b->fu = pss::BatchLaunch{};
    b->fx = pss::BatchLaunch{};
    b->fu_lds = b->fx_lds = 0;
    b->in_fu.assign(b->cls.size(), 0);
    b->in_fx.assign(b->cls.size(), 0);
    b->in_res.assign(b->cls.size(), 0);
    b->res.clear();
    int dev = 0, max_lds = 0;
    const bool lds_ok = hipGetDevice(&dev) == hipSuccess &&
                        hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
                        pss::resident_setup() == hipSuccess;
    for (size_t k = 0; k < b->cls.size(); ++k) {
        auto& cl = b->cls[k];
        pss_ctx* r = cl.rep;
        const int nmem = static_cast<int>(cl.idx.size());
        const bool plain = r->fields.size() == 1 && !r->plan.general;
        // whole lattices in LDS: one field whose products use only that field
        if (plain && b->resident && lds_ok && pss::resident_shape(r->n[0], r->n[1]) && r->geo.pu == 4 &&
            r->geo.px == 4 && r->geo.to == 1 && r->plan.nch <= 1 && r->plan.ng == r->plan.nch &&
            static_cast<int>(pss::resident_lds_bytes(r->n[0], r->n[1])) <= max_lds) {
            pss::ResidentLaunch rl{};
            rl.lx = r->n[0];
            rl.ly = r->n[1];
            rl.nmem = nmem;
            rl.members = cl.d_u;
            rl.plans = cl.d_plans;
            rl.tw_x = r->d_tw_x;
            rl.tw_y = r->d_tw_u;
            rl.geo = r->geo;
            b->res.push_back(rl);
            b->in_res[k] = 1;
            continue;
        }
        if (plain && r->geo.pu == 4 && r->geo.to == 1 && r->geo.tc * (r->lu / 4) == 256 && pss::batch_fused_len(r->lu) &&
            b->fu.ncls < pss::kMaxBatchClasses) {
            pss::BatchClass& C = b->fu.cls[b->fu.ncls++];
            C.L = r->lu;
            C.start = b->fu.total;
            C.nblk = r->geo.nublk;
            C.members = cl.d_u;
            C.plans = cl.d_plans;
            C.tw = r->d_tw_u;
            C.geo = r->geo;
            b->fu.total += nmem * C.nblk;
            // the fused update kernel's transforms are unpadded (its register budget)
            b->fu_lds = std::max(b->fu_lds, pss::update_lds_bytes(r->lu, 4, r->geo.tc, 1, 0));
            b->in_fu[k] = 1;
        }
        const int nx = r->n[0], ny = r->n[1];
        const int rbf = nx >= 64 ? 2048 / nx : 0;
        if (plain && r->plan.nch > 0 && r->plan.ng <= 1 && r->geo.px == 4 && pss::batch_fused_len(nx) && rbf >= 2 &&
            rbf <= ny && b->fx.ncls < pss::kMaxBatchClasses) {
            pss::BatchClass& C = b->fx.cls[b->fx.ncls++];
            C.L = nx;
            C.start = b->fx.total;
            C.nblk = ny / rbf;
            C.members = cl.d_x;
            C.plans = cl.d_plans;
            C.tw = r->d_tw_x;
            C.geo = r->geo;
            C.geo.rb = rbf;
            C.geo.rb_log2 = 0;
            while ((1 << C.geo.rb_log2) < rbf) ++C.geo.rb_log2;
            C.geo.nrowblk = ny / rbf;
            b->fx.total += nmem * C.nblk;
            b->fx_lds = std::max(b->fx_lds, pss::xrow_lds_bytes(nx, 4, rbf));
            b->in_fx[k] = 1;
        }
    }
}

int batch_launches_per_step(const pss_batch* b) {
    int n = (b->fu.ncls > 0) + (b->fx.ncls > 0);
    for (size_t k = 0; k < b->cls.size(); ++k) {
        if (b->in_res[k]) continue;
        if (!b->in_fu[k]) ++n;
        if (!b->in_fx[k] && b->cls[k].rep->plan.nch > 0) ++n;
    }
    return n;
}

pss_status batch_enqueue(pss_batch* b, int64_t k) {
    // classes with an x kernel move their members' counters on in the last
    // step's x launch, resident classes in their own launch; otherwise the
    // counter kernel moves every member's counter
    bool all_x = true;
    for (size_t c = 0; c < b->cls.size(); ++c) all_x = all_x && (b->in_res[c] || b->cls[c].rep->plan.nch > 0);
    for (const pss::ResidentLaunch& rl0 : b->res) {
        pss::ResidentLaunch rl = rl0;
        rl.nsteps = static_cast<int>(k);
        rl.advance = all_x ? 1 : 0;
        HIP_TRY(pss::launch_batch_resident(b->stream, rl));
    }
    for (int64_t i = 0; i < k; ++i) {
        const int64_t adv = (all_x && i == k - 1) ? k : 0;
        if (b->fu.ncls > 0) {
            pss::BatchLaunch bl = b->fu;
            bl.step_off = static_cast<int>(i);
            HIP_TRY(pss::launch_batch_update(b->stream, bl, b->fu_lds));
        }
        for (size_t c = 0; c < b->cls.size(); ++c) {
            if (b->in_fu[c] || b->in_res[c]) continue;
            auto& cl = b->cls[c];
            pss_ctx* r = cl.rep;
            pss::LaunchArgs a = args(r, static_cast<int>(i));
            a.stream = b->stream;
            a.members = cl.d_u;
            a.plans = cl.d_plans;
            a.nmem = static_cast<int>(cl.idx.size());
            HIP_TRY(pss::launch_update(pss::MODE_STEP, r->lu, static_cast<int>(r->fields.size()), a));
        }
        if (b->fx.ncls > 0) {
            pss::BatchLaunch bl = b->fx;
            bl.advance = adv;
            HIP_TRY(pss::launch_batch_xrow(b->stream, bl, b->fx_lds));
        }
        for (size_t c = 0; c < b->cls.size(); ++c) {
            auto& cl = b->cls[c];
            pss_ctx* r = cl.rep;
            if (b->in_fx[c] || b->in_res[c] || r->plan.nch == 0) continue;
            pss::LaunchArgs ax = xargs(r);
            ax.stream = b->stream;
            ax.members = cl.d_x;
            ax.plans = cl.d_plans;
            ax.nmem = static_cast<int>(cl.idx.size());
            ax.advance = adv;
            HIP_TRY(pss::launch_xrow(pss::MODE_STEP, r->n[0], r->plan.ng, ax));
        }
    }
    if (!all_x) HIP_TRY(pss::launch_advance_many(b->stream, b->d_ctrs, static_cast<int>(b->mem.size()), k));
    return PSS_OK;
}

// time `reps` back-to-back fused launches of one phase (HIP events on the batch stream)
pss_status batch_time_fused(pss_batch* b, int32_t which, int32_t reps, double* ms, double* bytes) {
    const pss::BatchLaunch& fl = which == 0 ? b->fu : b->fx;
    if (fl.ncls == 0) return fail(PSS_E_INVAL, "the batch has no fused %s launch", which == 0 ? "update" : "x");
    std::vector<int> members;
    const std::vector<char>& in = which == 0 ? b->in_fu : b->in_fx;
    double total = 0;
    for (size_t k = 0; k < b->cls.size(); ++k) {
        if (!in[k]) continue;
        members.insert(members.end(), b->cls[k].idx.begin(), b->cls[k].idx.end());
        double one = 0;
        if (pss_status s = pss_kernel_bytes(b->cls[k].rep, which, &one)) return s;
        total += one * static_cast<double>(b->cls[k].idx.size());
    }
    if (pss_status s = batch_order_before(b, members)) return s;
    if (pss_status s = batch_refresh_plans(b)) return s;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, b->stream));
    for (int r = 0; r < reps; ++r) {
        if (which == 0)
            HIP_TRY(pss::launch_batch_update(b->stream, b->fu, b->fu_lds));
        else
            HIP_TRY(pss::launch_batch_xrow(b->stream, b->fx, b->fx_lds));
    }
    HIP_TRY(hipEventRecord(e1, b->stream));
    HIP_TRY(hipEventSynchronize(e1));
    float t = 0;
    HIP_TRY(hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = static_cast<double>(t) / reps;
    if (bytes) *bytes = total;
    for (int i : members) {  // repeated launches leave the channels stale and change the states
        b->mem[i]->dirty = true;
        ++b->mem[i]->state_gen;
    }
    return batch_order_after(b, members);
}

// time one launch of `reps` steps of every resident class (HIP events on the
// batch stream): milliseconds and HBM bytes per step
pss_status batch_time_resident(pss_batch* b, int32_t reps, double* ms, double* bytes) {
    if (b->res.empty()) return fail(PSS_E_INVAL, "the batch has no LDS-resident class");
    std::vector<int> members;
    double total = 0;
    for (size_t k = 0; k < b->cls.size(); ++k) {
        if (!b->in_res[k]) continue;
        members.insert(members.end(), b->cls[k].idx.begin(), b->cls[k].idx.end());
        // state and channel array in and out once per launch
        total += 16.0 * static_cast<double>(b->cls[k].rep->sites()) * static_cast<double>(b->cls[k].idx.size());
    }
    if (pss_status s = batch_order_before(b, members)) return s;
    if (pss_status s = batch_refresh_plans(b)) return s;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, b->stream));
    for (const pss::ResidentLaunch& rl0 : b->res) {
        pss::ResidentLaunch rl = rl0;
        rl.nsteps = reps;
        rl.advance = 0;
        HIP_TRY(pss::launch_batch_resident(b->stream, rl));
    }
    HIP_TRY(hipEventRecord(e1, b->stream));
    HIP_TRY(hipEventSynchronize(e1));
    float t = 0;
    HIP_TRY(hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = static_cast<double>(t) / reps;
    if (bytes) *bytes = total / reps;
    for (int i : members) {  // the states moved on without their counters
        b->mem[i]->dirty = true;
        ++b->mem[i]->state_gen;
    }
    return batch_order_after(b, members);
}

pss_status batch_graph_for(pss_batch* b, int64_t k, hipGraphExec_t* out) {
    auto it = b->graphs.find(k);
    if (it != b->graphs.end()) {
        *out = it->second;
        return PSS_OK;
    }
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal));
    pss_status st = batch_enqueue(b, k);
    hipError_t e = hipStreamEndCapture(b->stream, &g);
    if (st) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    HIP_TRY(e);
    hipGraphExec_t ex = nullptr;
    e = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIP_TRY(e);
    b->graphs[k] = ex;
    *out = ex;
    return PSS_OK;
}

// unpack the state of one field (packed columns, slot form on packed lines)
// into the canonical half spectrum
void unpack_half(const pss_ctx* c, const std::vector<float2>& S, float* out) {
    const int nx = c->n[0], ny = c->n[1], tc = c->geo.tc, ntile = c->geo.ntile;
    const int nz = c->ndim == 3 ? c->n[2] : 1;
    const int nh = nx / 2 + 1;
    auto put = [&](int z, int y, int kx, double re, double im) {
        const size_t i = 2 * ((static_cast<size_t>(z) * ny + y) * nh + kx);
        out[i] = static_cast<float>(re);
        out[i + 1] = static_cast<float>(im);
    };
    auto at = [&](int col, int y, int z) {
        if (c->ndim == 2) return S[(static_cast<size_t>(col / tc) * ny + y) * tc + col % tc];
        return S[((static_cast<size_t>(y) * ntile + col / tc) * nz + z) * tc + col % tc];
    };
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int col = 1; col < nx / 2; ++col) {
                const float2 v = at(col, y, z);
                put(z, y, col, v.x, v.y);
            }
    // planes kx = 0 and kx = Nx/2: collect what is stored, then fill the rest
    // by Hermitian symmetry phi(kx0, -y, -z) = conj phi(kx0, y, z)
    const size_t np = static_cast<size_t>(ny) * nz;
    std::vector<std::complex<double>> P0(np), PN(np);
    std::vector<char> k0(np, 0), kn(np, 0);
    auto idx = [&](int y, int z) { return static_cast<size_t>(z) * ny + y; };
    auto slots = [&](int L, auto get, auto set0, auto setn) {  // packed line of length L
        for (int u = 0; u < L; ++u) {
            const float2 v = get(u);
            if (u == 0 || u == L / 2) {
                set0(u, std::complex<double>(v.x, 0));
                setn(u, std::complex<double>(v.y, 0));
            } else if (u < L / 2) {
                set0(u, std::complex<double>(v.x, v.y));
            } else {
                setn(L - u, std::complex<double>(v.x, v.y));
            }
        }
    };
    if (c->ndim == 2) {
        slots(
            ny, [&](int u) { return at(0, u, 0); },
            [&](int y, std::complex<double> v) { P0[idx(y, 0)] = v; k0[idx(y, 0)] = 1; },
            [&](int y, std::complex<double> v) { PN[idx(y, 0)] = v; kn[idx(y, 0)] = 1; });
    } else {
        for (int o = 0; o < ny; ++o) {
            if (o == 0 || o == ny / 2) {
                slots(
                    nz, [&](int u) { return at(0, o, u); },
                    [&](int z, std::complex<double> v) { P0[idx(o, z)] = v; k0[idx(o, z)] = 1; },
                    [&](int z, std::complex<double> v) { PN[idx(o, z)] = v; kn[idx(o, z)] = 1; });
            } else {
                for (int z = 0; z < nz; ++z) {
                    const float2 v = at(0, o, z);
                    if (o < ny / 2) {
                        P0[idx(o, z)] = {v.x, v.y};
                        k0[idx(o, z)] = 1;
                    } else {
                        PN[idx(ny - o, z)] = {v.x, v.y};
                        kn[idx(ny - o, z)] = 1;
                    }
                }
            }
        }
    }
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y) {
            const size_t i = idx(y, z), j = idx((ny - y) & (ny - 1), (nz - z) & (nz - 1));
            const std::complex<double> a = k0[i] ? P0[i] : std::conj(P0[j]);
            const std::complex<double> b = kn[i] ? PN[i] : std::conj(PN[j]);
            put(z, y, 0, a.real(), a.imag());
            put(z, y, nx / 2, b.real(), b.imag());
        }
}

struct SaveHeader {
    char magic[8];
    int32_t ndim, nf;
    int32_t n[3];
    int32_t tc;
    int64_t step;
};

}  // namespace

extern "C" {

const char* pss_last_error(void) { return g_err.c_str(); }

pss_status pss_lattice_create(pss_ctx** out, int32_t ndim, const int64_t n[3], const double dx[3], double dt) {
    if (!out || !n || !dx) return fail(PSS_E_INVAL, "null argument");
    *out = nullptr;
    if (ndim < 1 || ndim > 3) return fail(PSS_E_UNSUPPORTED, "ndim must be 1, 2 or 3 (got %d)", ndim);
    if (!(dt > 0) || !std::isfinite(dt)) return fail(PSS_E_INVAL, "dt must be positive");
    int64_t total = 1;
    for (int i = 0; i < ndim; ++i) {
        if (!(dx[i] > 0) || !std::isfinite(dx[i])) return fail(PSS_E_INVAL, "dx[%d] must be positive", i);
        // sizes are powers of two or mixed-radix lengths 2^a 3^b 5^c (a >= 1)
        pss::MrPlan mr{};
        const bool mixed = n[i] >= 8 && n[i] <= 4096 && pss::mr_plan(static_cast<int>(n[i]), &mr);
        if ((!is_pow2(n[i]) && !mixed) || n[i] < 8 || n[i] > 4096)
            return fail(PSS_E_UNSUPPORTED, "n[%d] = %lld is not an even 2^a 3^b 5^c in [8, 4096]", i,
                        static_cast<long long>(n[i]));
        total *= n[i];
    }
    if (total > (int64_t(1) << 31)) return fail(PSS_E_UNSUPPORTED, "more than 2^31 sites");
    pss_ctx* c = new pss_ctx();
    c->ndim = ndim;
    for (int i = 0; i < ndim; ++i) {
        c->n[i] = static_cast<int>(n[i]);
        c->dx[i] = dx[i];
    }
    c->mixed = ndim >= 2 && (!is_pow2(n[0]) || !is_pow2(n[1]) || (ndim == 3 && !is_pow2(n[2])));
    c->dt = dt;
    const char* dbg = std::getenv("PSS_DEBUG_SYNC");
    c->debug_sync = dbg && *dbg && std::strcmp(dbg, "0") != 0;
    *out = c;
    return PSS_OK;
}

pss_status pss_lattice_destroy(pss_ctx* c) {
    if (!c) return PSS_OK;
    if (c->batches > 0) return fail(PSS_E_STATE, "lattice is held by %d batch(es); destroy them first", c->batches);
    if (c->tapes > 0) return fail(PSS_E_STATE, "an adjoint tape holds this lattice; destroy it first");
    free_device(c);
    delete c;
    return PSS_OK;
}

pss_status pss_field_declare(pss_ctx* c, const char* name, int32_t dynamic, int32_t* field_id) {
    if (pss_status s = check_ctx(c)) return s;
    if (c->planned) return fail(PSS_E_STATE, "fields cannot be added after the plan is built");
    if (!name || !*name || std::strlen(name) > 63) return fail(PSS_E_INVAL, "field name must have 1..63 characters");
    for (const Field& f : c->fields)
        if (f.name == name) return fail(PSS_E_INVAL, "field '%s' already declared", name);
    for (const std::string& f : c->interms)
        if (f == name) return fail(PSS_E_INVAL, "field '%s' already declared", name);
    if (dynamic) {
        if (static_cast<int>(c->fields.size()) >= PSS_MAXF)
            return fail(PSS_E_UNSUPPORTED, "at most %d dynamic fields", PSS_MAXF);
        Field f;
        f.name = name;
        c->fields.push_back(f);
        c->ids.push_back(static_cast<int>(c->fields.size()) - 1);
    } else {
        if (static_cast<int>(c->interms.size()) >= PSS_MAXI)
            return fail(PSS_E_UNSUPPORTED, "at most %d intermediate fields", PSS_MAXI);
        c->interms.push_back(name);
        c->ids.push_back(PSS_MAXF + static_cast<int>(c->interms.size()) - 1);
    }
    if (field_id) *field_id = static_cast<int32_t>(c->ids.size() - 1);
    return PSS_OK;
}

pss_status pss_field_find(pss_ctx* c, const char* name, int32_t* field_id, int32_t* dynamic) {
    if (pss_status s = check_ctx(c)) return s;
    if (!name) return fail(PSS_E_INVAL, "null name");
    for (size_t id = 0; id < c->ids.size(); ++id) {
        const int code = c->ids[id];
        const std::string& nm = is_interm(code) ? c->interms[code - PSS_MAXF] : c->fields[code].name;
        if (nm == name) {
            if (field_id) *field_id = static_cast<int32_t>(id);
            if (dynamic) *dynamic = is_interm(code) ? 0 : 1;
            return PSS_OK;
        }
    }
    return fail(PSS_E_INVAL, "no field named '%s'", name);
}

pss_status pss_param_set(pss_ctx* c, const char* name, double value) {
    if (pss_status s = check_ctx(c)) return s;
    if (!name || !*name || std::strlen(name) > 63) return fail(PSS_E_INVAL, "parameter name must have 1..63 characters");
    if (!std::isfinite(value)) return fail(PSS_E_INVAL, "non-finite parameter value");
    c->params[name] = value;
    return PSS_OK;
}

pss_status pss_param_get(pss_ctx* c, const char* name, double* value) {
    if (pss_status s = check_ctx(c)) return s;
    if (!name || !value) return fail(PSS_E_INVAL, "null argument");
    auto it = c->params.find(name);
    if (it == c->params.end()) return fail(PSS_E_INVAL, "no parameter named '%s'", name);
    *value = it->second;
    return PSS_OK;
}

pss_status pss_term_add(pss_ctx* c, int32_t target, int32_t implicit, const pss_qmono* op, int32_t n_mono,
                        const int32_t* factor_fields, const int32_t* factor_powers, int32_t n_factors,
                        int32_t* term_id) {
    if (pss_status s = check_ctx(c)) return s;
    if (c->planned) return fail(PSS_E_STATE, "terms cannot be added after the plan is built");
    const int tcode = field_code(c, target);
    if (tcode < 0) return fail(PSS_E_INVAL, "target field %d out of range", target);
    if (pss_status s = check_ops(op, n_mono, false)) return s;
    if (n_factors < 1 || n_factors > 4 || !factor_fields || !factor_powers)
        return fail(PSS_E_INVAL, "a term needs 1..4 factors");
    if (static_cast<int>(c->terms.size()) >= PSS_MAXT) return fail(PSS_E_UNSUPPORTED, "at most %d terms", PSS_MAXT);
    Term t;
    t.target = tcode;
    t.implicit = implicit != 0;
    t.op = to_monos(op, n_mono);
    for (int i = 0; i < n_factors; ++i) {
        const int code = field_code(c, factor_fields[i]);
        if (code < 0) return fail(PSS_E_INVAL, "factor field %d out of range", factor_fields[i]);
        if (factor_powers[i] < 1 || factor_powers[i] > PSS_MAXPOW)
            return fail(PSS_E_INVAL, "factor powers must lie in [1, %d]", PSS_MAXPOW);
        t.factors.push_back({code, factor_powers[i]});
    }
    if (t.implicit && !(n_factors == 1 && factor_fields[0] == target && factor_powers[0] == 1))
        return fail(PSS_E_INVAL, "an implicit term must be linear in its own field (op * field)");
    if (is_interm(tcode) && !t.implicit &&
        !(n_factors == 1 && factor_powers[0] == 1 && !is_interm(t.factors[0].first)))
        return fail(PSS_E_UNSUPPORTED,
                    "an explicit term of an intermediate field must be one dynamic field to the first power");
    int total = 0;
    for (auto& fp : t.factors) total += fp.second;
    if (total > PSS_MAXPOW) return fail(PSS_E_INVAL, "total order above %d", PSS_MAXPOW);
    c->terms.push_back(t);
    if (term_id) *term_id = static_cast<int32_t>(c->terms.size() - 1);
    return PSS_OK;
}

pss_status pss_term_info(pss_ctx* c, int32_t term_id, int32_t* target, int32_t* implicit, pss_qmono* op,
                         int32_t* n_mono, int32_t* factor_fields, int32_t* factor_powers, int32_t* n_factors) {
    if (pss_status s = check_ctx(c)) return s;
    if (term_id < 0 || term_id >= static_cast<int>(c->terms.size())) return fail(PSS_E_INVAL, "bad term id");
    const Term& t = c->terms[term_id];
    auto declared = [&](int code) {
        for (size_t id = 0; id < c->ids.size(); ++id)
            if (c->ids[id] == code) return static_cast<int32_t>(id);
        return int32_t{-1};
    };
    if (target) *target = declared(t.target);
    if (implicit) *implicit = t.implicit ? 1 : 0;
    if (n_mono) *n_mono = static_cast<int32_t>(t.op.size());
    if (op)
        for (size_t i = 0; i < t.op.size(); ++i) {
            op[i].coef = t.op[i].coef;
            op[i].q2_pow = t.op[i].q2;
            op[i].invq_pow = t.op[i].invq;
            for (int k = 0; k < 3; ++k) op[i].iq_pow[k] = t.op[i].iq[k];
        }
    if (n_factors) *n_factors = static_cast<int32_t>(t.factors.size());
    for (size_t i = 0; i < t.factors.size(); ++i) {
        if (factor_fields) factor_fields[i] = declared(t.factors[i].first);
        if (factor_powers) factor_powers[i] = t.factors[i].second;
    }
    return PSS_OK;
}

pss_status pss_term_count(pss_ctx* c, int32_t* count) {
    if (pss_status s = check_ctx(c)) return s;
    if (!count) return fail(PSS_E_INVAL, "null output");
    *count = static_cast<int32_t>(c->terms.size());
    return PSS_OK;
}

pss_status pss_term_set_coef(pss_ctx* c, int32_t term_id, int32_t mono, double coef) {
    if (pss_status s = check_ctx(c)) return s;
    if (term_id < 0 || term_id >= static_cast<int>(c->terms.size())) return fail(PSS_E_INVAL, "bad term id");
    Term& t = c->terms[term_id];
    if (mono < 0 || mono >= static_cast<int>(t.op.size())) return fail(PSS_E_INVAL, "bad monomial index");
    if (!std::isfinite(coef)) return fail(PSS_E_INVAL, "non-finite coefficient");
    const double old = t.op[mono].coef;
    t.op[mono].coef = coef;
    if (t.implicit) {
        if (pss_status s = validate(c)) {
            t.op[mono].coef = old;
            return s;
        }
    }
    if (!c->planned) return PSS_OK;
    // recompile the coefficients (the structure is unchanged), and rebuild the
    // channel arrays of the next step from the current state
    const pss::DevPlan keep = c->plan;
    if (pss_status s = build_plan(c)) {
        t.op[mono].coef = old;
        c->plan = keep;
        return s;
    }
    c->dirty = true;
    return upload_plan(c);
}

pss_status pss_noise_set(pss_ctx* c, int32_t field, const pss_qmono* D, int32_t n_mono) {
    if (pss_status s = check_ctx(c)) return s;
    int fd = 0;
    if (pss_status s = dyn_field(c, field, &fd)) return s;
    if (pss_status s = check_ops(D, n_mono, true)) return s;
    std::vector<Mono> nm = to_monos(D, n_mono);
    Field& fl = c->fields[fd];
    if (!c->planned) {
        fl.noisy = true;
        fl.noise = nm;
        return PSS_OK;
    }
    // after planning: new coefficients of the same monomials only
    bool same = fl.noisy && fl.noise.size() == nm.size();
    for (size_t i = 0; same && i < nm.size(); ++i)
        same = fl.noise[i].q2 == nm[i].q2 && fl.noise[i].invq == nm[i].invq && fl.noise[i].iq[0] == nm[i].iq[0] &&
               fl.noise[i].iq[1] == nm[i].iq[1] && fl.noise[i].iq[2] == nm[i].iq[2];
    if (!same) return fail(PSS_E_STATE, "after the plan is built only the coefficients of a noise operator can change");
    const std::vector<Mono> old = fl.noise;
    const pss::DevPlan keep = c->plan;
    fl.noise = nm;
    pss_status st = validate(c);
    if (!st) st = build_plan(c);
    if (st) {
        fl.noise = old;
        c->plan = keep;
        return st;
    }
    return upload_plan(c);
}

pss_status pss_frame_set(pss_ctx* c, int32_t field, const int64_t* sites, const float* values, int64_t n) {
    if (pss_status s = check_ctx(c)) return s;
    int fd = 0;
    if (pss_status s = dyn_field(c, field, &fd)) return s;
    if (n < 0 || (n > 0 && (!sites || !values))) return fail(PSS_E_INVAL, "bad frame arrays");
    if (n > c->sites()) return fail(PSS_E_INVAL, "more frame sites than lattice sites");
    if (c->batches > 0) return fail(PSS_E_STATE, "a batch holds this lattice (batched steps apply no frames)");
    if (c->tapes > 0) return fail(PSS_E_STATE, "an adjoint tape holds this lattice");
    std::vector<int2> fr(static_cast<size_t>(n));
    for (int64_t i = 0; i < n; ++i) {
        if (sites[i] < 0 || sites[i] >= c->sites()) return fail(PSS_E_INVAL, "frame site %lld off the lattice",
                                                                  static_cast<long long>(sites[i]));
        if (!std::isfinite(values[i])) return fail(PSS_E_INVAL, "non-finite frame value");
        int bits;
        std::memcpy(&bits, &values[i], sizeof(bits));
        fr[static_cast<size_t>(i)] = make_int2(static_cast<int>(sites[i]), bits);
    }
    if (c->frames.size() < c->fields.size()) c->frames.resize(c->fields.size());
    c->frames[fd] = std::move(fr);
    if (!c->planned) return PSS_OK;
    // on the device now; the step sequence changes in 2D and 3D
    if (pss_status s = begin_work(c)) return s;
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
    if (pss_status s = upload_frames(c)) return s;
    return upload_plan(c);
}

pss_status pss_seed_set(pss_ctx* c, uint64_t seed) {
    if (pss_status s = check_ctx(c)) return s;
    c->seed = seed;
    if (c->planned) {
        c->plan.key0 = static_cast<uint32_t>(seed & 0xffffffffu);
        c->plan.key1 = static_cast<uint32_t>(seed >> 32);
        return upload_plan(c);
    }
    return PSS_OK;
}

pss_status pss_dealias_set(pss_ctx* c, int32_t rule, int32_t shape) {
    if (pss_status s = check_ctx(c)) return s;
    if (c->planned) return fail(PSS_E_STATE, "de-aliasing cannot be changed after the plan is built");
    if (rule < 0 || rule > 2 || shape < 0 || shape > 1) return fail(PSS_E_INVAL, "bad de-aliasing rule or shape");
    c->rule = rule;
    c->shape = shape;
    return PSS_OK;
}

pss_status pss_stream_set(pss_ctx* c, void* stream) {
    if (pss_status s = check_ctx(c)) return s;
    // a batch launches on its first member's stream and orders itself
    // against the others' streams: they must stay what they were
    if (c->batches > 0)
        return fail(PSS_E_STATE, "lattice is held by %d batch(es); destroy them before changing its stream",
                    c->batches);
    if (c->tapes > 0) return fail(PSS_E_STATE, "an adjoint tape holds this lattice; destroy it first");
    if (c->planned && c->stream) HIP_TRY(hipStreamSynchronize(c->stream));
    if (c->own_stream && c->stream) {
        (void)hipStreamDestroy(c->stream);
        c->own_stream = false;
        c->stream = nullptr;
    }
    for (auto& kv : c->graphs) (void)hipGraphExecDestroy(kv.second);
    c->graphs.clear();
    c->stream = static_cast<hipStream_t>(stream);
    if (!c->stream && c->planned) {
        HIP_TRY(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        c->own_stream = true;
    }
    return PSS_OK;
}

pss_status pss_tuning_set(pss_ctx* c, const char* key, int64_t value) {
    if (pss_status s = check_ctx(c)) return s;
    if (c->planned) return fail(PSS_E_STATE, "the launch geometry is fixed once the plan is built");
    static const char* keys[] = {"tc", "to", "tz", "rb", "pu", "px", "py"};
    if (!key) return fail(PSS_E_INVAL, "null key");
    for (const char* k : keys)
        if (std::strcmp(k, key) == 0) {
            if (value <= 0) {
                c->tune.erase(key);
            } else {
                c->tune[key] = value;
            }
            return PSS_OK;
        }
    return fail(PSS_E_INVAL, "unknown tuning key '%s'", key);
}

pss_status pss_tuning_get(pss_ctx* c, const char* key, int64_t* value) {
    if (pss_status s = check_ctx(c)) return s;
    if (!key || !value) return fail(PSS_E_INVAL, "null argument");
    if (pss_status s = materialize(c)) return s;
    const pss::Geo& g = c->geo;
    const std::pair<const char*, int> vals[] = {{"tc", g.tc}, {"to", g.to}, {"tz", g.tz}, {"rb", g.rb},
                                                {"pu", g.pu}, {"px", g.px}, {"py", g.py}};
    for (auto& kv : vals)
        if (std::strcmp(kv.first, key) == 0) {
            *value = kv.second;
            return PSS_OK;
        }
    return fail(PSS_E_INVAL, "unknown tuning key '%s'", key);
}

pss_status pss_validate(pss_ctx* c) {
    if (pss_status s = check_ctx(c)) return s;
    return validate(c);
}

pss_status pss_field_upload(pss_ctx* c, int32_t field, const float* real, int32_t on_device) {
    if (pss_status s = check_ctx(c)) return s;
    if (!real) return fail(PSS_E_INVAL, "null array");
    if (pss_status s = materialize(c)) return s;
    int fd = 0;
    if (pss_status s = dyn_field(c, field, &fd)) return s;
    if (pss_status s_bw = begin_work(c)) return s_bw;
    const size_t bytes = sizeof(float) * static_cast<size_t>(c->sites());
    HIP_TRY(hipMemcpyAsync(c->d_real, real, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                           c->stream));
    if (pss_status s = forward_to_state(c, fd)) return s;
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->dirty = true;
    ++c->state_gen;
    return clear_nonfinite(c);
}

pss_status pss_field_init_uniform(pss_ctx* c, int32_t field, double lo, double hi) {
    if (pss_status s = check_ctx(c)) return s;
    if (!std::isfinite(lo) || !std::isfinite(hi)) return fail(PSS_E_INVAL, "non-finite bounds");
    if (pss_status s = materialize(c)) return s;
    int fd = 0;
    if (pss_status s = dyn_field(c, field, &fd)) return s;
    if (pss_status s_bw = begin_work(c)) return s_bw;
    // keyed by the declared field number, as the noise is
    HIP_TRY(pss::launch_init_uniform(c->stream, c->d_real, c->sites(), static_cast<uint32_t>(field),
                                     c->plan.key0, c->plan.key1, lo, hi));
    if (pss_status s = forward_to_state(c, fd)) return s;
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->dirty = true;
    ++c->state_gen;
    return clear_nonfinite(c);
}

pss_status pss_field_download(pss_ctx* c, int32_t field, float* real, int32_t on_device) {
    if (pss_status s = check_ctx(c)) return s;
    if (!real) return fail(PSS_E_INVAL, "null array");
    if (pss_status s = materialize(c)) return s;
    const int code = field_code(c, field);
    if (code < 0) return fail(PSS_E_INVAL, "bad field");
    if (pss_status s_bw = begin_work(c)) return s_bw;
    if (is_interm(code)) {
        if (pss_status s = interm_to_real(c, code - PSS_MAXF)) return s;
    } else if (pss_status s = state_to_real(c, code)) {
        return s;
    }
    const size_t bytes = sizeof(float) * static_cast<size_t>(c->sites());
    HIP_TRY(hipMemcpyAsync(real, c->d_real, bytes, on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                           c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    return PSS_OK;
}

pss_status pss_spectrum_download(pss_ctx* c, int32_t field, float* half, int32_t on_device) {
    if (pss_status s = check_ctx(c)) return s;
    if (!half) return fail(PSS_E_INVAL, "null array");
    if (pss_status s = materialize(c)) return s;
    int fd = 0;
    if (pss_status s = dyn_field(c, field, &fd)) return s;
    if (pss_status s_bw = begin_work(c)) return s_bw;
    std::vector<float2> S(static_cast<size_t>(c->packed()));
    HIP_TRY(hipMemcpyAsync(S.data(), c->d_state[fd], sizeof(float2) * S.size(), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    const size_t nout = static_cast<size_t>(c->n[1]) * (c->ndim == 3 ? c->n[2] : 1) * (c->n[0] / 2 + 1) * 2;
    std::vector<float> h(nout);
    if (c->ndim == 1) {  // modes 0 .. Nx/2 of the full spectrum
        for (int k = 0; k <= c->n[0] / 2; ++k) {
            h[2 * k] = S[k].x;
            h[2 * k + 1] = S[k].y;
        }
    } else if (c->mixed) {  // kx = 0 .. Nx/2 of the full spectrum, every (ky, kz)
        const int nx = c->n[0], nh = nx / 2 + 1;
        const size_t rows = static_cast<size_t>(c->n[1]) * (c->ndim == 3 ? c->n[2] : 1);
        for (size_t y = 0; y < rows; ++y)
            for (int k = 0; k < nh; ++k) {
                const float2 v = S[y * nx + k];
                h[2 * (y * nh + k)] = v.x;
                h[2 * (y * nh + k) + 1] = v.y;
            }
    } else {
        unpack_half(c, S, h.data());
    }
    if (on_device) {
        HIP_TRY(hipMemcpy(half, h.data(), sizeof(float) * nout, hipMemcpyHostToDevice));
    } else {
        std::memcpy(half, h.data(), sizeof(float) * nout);
    }
    return PSS_OK;
}

pss_status pss_step(pss_ctx* c, int64_t nsteps) {
    if (pss_status s = check_ctx(c)) return s;
    if (nsteps < 0) return fail(PSS_E_INVAL, "negative step count");
    if (nsteps == 0) return PSS_OK;
    if (pss_status s = materialize(c)) return s;
    if (pss_status s_bw = begin_work(c)) return s_bw;
    if (c->dirty) {
        if (pss_status s = prologue(c)) return s;
        if (pss_status s = debug_check(c, "products of the state", c->steps_taken)) return s;
    }
    if (c->debug_sync) {
        // the same kernels, enqueued one by one and checked after each
        for (int64_t i = 0; i < nsteps; ++i) {
            if (pss_status s = enqueue_steps(c, 1)) {
                ++c->state_gen;
                return s;
            }
            ++c->steps_taken;
        }
        ++c->state_gen;
        return PSS_OK;
    }
    int64_t left = nsteps;
    while (left > 0) {
        const int64_t k = std::min(left, kGraphSteps);
        hipGraphExec_t ex = nullptr;
        if (pss_status s = graph_for(c, k, &ex)) return s;
        HIP_TRY(hipGraphLaunch(ex, c->stream));
        left -= k;
    }
    c->steps_taken += nsteps;
    ++c->state_gen;
    return PSS_OK;
}

pss_status pss_step_prepare(pss_ctx* c, int64_t nsteps) {
    if (pss_status s = check_ctx(c)) return s;
    if (nsteps < 0) return fail(PSS_E_INVAL, "negative step count");
    if (pss_status s = materialize(c)) return s;
    // the chunk lengths pss_step(nsteps) replays: full chunks and the remainder
    const int64_t lens[2] = {std::min(nsteps, kGraphSteps), nsteps % kGraphSteps};
    for (int64_t k : lens) {
        if (k <= 0) continue;
        hipGraphExec_t ex = nullptr;
        if (pss_status s = graph_for(c, k, &ex)) return s;
    }
    return PSS_OK;
}

pss_status pss_step_index(pss_ctx* c, int64_t* out) {
    if (pss_status s = check_ctx(c)) return s;
    if (!out) return fail(PSS_E_INVAL, "null output");
    *out = c->steps_taken;
    return PSS_OK;
}

pss_status pss_sync(pss_ctx* c) {
    if (pss_status s = check_ctx(c)) return s;
    if (c->planned)
        if (pss_status s = begin_work(c)) return s;
    if (c->stream) HIP_TRY(hipStreamSynchronize(c->stream));
    return take_nonfinite(c);
}

pss_status pss_state_size(pss_ctx* c, size_t* bytes) {
    if (pss_status s = check_ctx(c)) return s;
    if (!bytes) return fail(PSS_E_INVAL, "null output");
    *bytes = sizeof(SaveHeader) + c->fields.size() * sizeof(float2) * static_cast<size_t>(c->packed());
    return PSS_OK;
}

pss_status pss_field_state_bytes(pss_ctx* c, int32_t field, size_t* bytes) {
    if (pss_status s = check_ctx(c)) return s;
    if (!bytes) return fail(PSS_E_INVAL, "null output");
    int fd = 0;
    if (pss_status s = dyn_field(c, field, &fd)) return s;
    *bytes = sizeof(float2) * static_cast<size_t>(c->packed());
    return PSS_OK;
}

pss_status pss_field_bind(pss_ctx* c, int32_t field, void* device_ptr, size_t bytes) {
    if (pss_status s = check_ctx(c)) return s;
    int fd = 0;
    if (pss_status s = dyn_field(c, field, &fd)) return s;
    if (c->planned) return fail(PSS_E_STATE, "bind before the plan is built (the state is already allocated)");
    if (!device_ptr) return fail(PSS_E_INVAL, "null memory");
    if (reinterpret_cast<uintptr_t>(device_ptr) % alignof(float2) != 0)
        return fail(PSS_E_INVAL, "memory must be %zu-byte aligned", alignof(float2));
    const size_t need = sizeof(float2) * static_cast<size_t>(c->packed());
    if (bytes < need) return fail(PSS_E_INVAL, "the state of field %d needs %zu bytes (got %zu)", field, need, bytes);
    c->bound[fd] = device_ptr;
    c->bound_bytes[fd] = bytes;
    return PSS_OK;
}

pss_status pss_state_changed(pss_ctx* c) {
    if (pss_status s = check_ctx(c)) return s;
    c->dirty = true;
    ++c->state_gen;
    return PSS_OK;
}

pss_status pss_state_save(pss_ctx* c, void* dst, size_t bytes) {
    if (pss_status s = check_ctx(c)) return s;
    size_t need = 0;
    pss_state_size(c, &need);
    if (!dst || bytes < need) return fail(PSS_E_INVAL, "state buffer needs %zu bytes", need);
    if (pss_status s = materialize(c)) return s;
    if (pss_status s_bw = begin_work(c)) return s_bw;
    SaveHeader h{};
    std::memcpy(h.magic, "PSSSTAT1", 8);
    h.ndim = c->ndim;
    h.nf = static_cast<int32_t>(c->fields.size());
    for (int i = 0; i < 3; ++i) h.n[i] = c->n[i];
    h.tc = c->geo.tc;
    h.step = c->steps_taken;
    std::memcpy(dst, &h, sizeof(h));
    char* p = static_cast<char*>(dst) + sizeof(h);
    const size_t fb = sizeof(float2) * static_cast<size_t>(c->packed());
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (size_t f = 0; f < c->fields.size(); ++f) HIP_TRY(hipMemcpy(p + f * fb, c->d_state[f], fb, hipMemcpyDeviceToHost));
    return PSS_OK;
}

pss_status pss_state_load(pss_ctx* c, const void* src, size_t bytes) {
    if (pss_status s = check_ctx(c)) return s;
    size_t need = 0;
    pss_state_size(c, &need);
    if (!src || bytes < need) return fail(PSS_E_INVAL, "state buffer needs %zu bytes", need);
    if (pss_status s = materialize(c)) return s;
    if (pss_status s_bw = begin_work(c)) return s_bw;
    SaveHeader h;
    std::memcpy(&h, src, sizeof(h));
    if (std::memcmp(h.magic, "PSSSTAT1", 8) != 0 || h.ndim != c->ndim || h.nf != static_cast<int>(c->fields.size()) ||
        h.n[0] != c->n[0] || h.n[1] != c->n[1] || h.n[2] != c->n[2] || h.tc != c->geo.tc)
        return fail(PSS_E_INVAL, "state buffer does not match this lattice");
    const char* p = static_cast<const char*>(src) + sizeof(h);
    const size_t fb = sizeof(float2) * static_cast<size_t>(c->packed());
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (size_t f = 0; f < c->fields.size(); ++f) HIP_TRY(hipMemcpy(c->d_state[f], p + f * fb, fb, hipMemcpyHostToDevice));
    const uint64_t st = static_cast<uint64_t>(h.step);
    HIP_TRY(hipMemcpy(c->d_step, &st, sizeof(st), hipMemcpyHostToDevice));
    c->steps_taken = h.step;
    c->dirty = true;
    ++c->state_gen;
    if (pss_status s = clear_nonfinite(c)) return s;
    return PSS_OK;
}

pss_status pss_mass(pss_ctx* c, int32_t field, double* mass) {
    if (pss_status s = check_ctx(c)) return s;
    if (!mass) return fail(PSS_E_INVAL, "null output");
    if (pss_status s = materialize(c)) return s;
    int fd = 0;
    if (pss_status s = dyn_field(c, field, &fd)) return s;
    if (pss_status s_bw = begin_work(c)) return s_bw;
    float2 v;
    HIP_TRY(hipMemcpyAsync(&v, c->d_state[fd], sizeof(v), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    *mass = static_cast<double>(v.x);  // Re of phi_hat(0) + i phi_hat(Nx/2, 0)
    return PSS_OK;
}

pss_status pss_structure_factor(pss_ctx* c, int32_t field, double* S, int64_t* counts, int32_t n_shells) {
    if (pss_status s = check_ctx(c)) return s;
    if (!S || !counts) return fail(PSS_E_INVAL, "null output");
    if (pss_status s = materialize(c)) return s;
    int fd = 0;
    if (pss_status s = dyn_field(c, field, &fd)) return s;
    if (pss_status s_bw = begin_work(c)) return s_bw;
    const int nmin = c->ndim == 3 ? std::min(std::min(c->n[0], c->n[1]), c->n[2])
                                  : (c->ndim == 2 ? std::min(c->n[0], c->n[1]) : c->n[0]);
    const int ns = nmin / 2;  // shells j = 1 .. ns-1
    if (n_shells != ns - 1) return fail(PSS_E_INVAL, "n_shells must be %d", ns - 1);
    if (!c->d_shell_acc) HIP_TRY(hipMalloc(&c->d_shell_acc, sizeof(unsigned long long) * pss::kShellWords * ns));
    HIP_TRY(hipMemsetAsync(c->d_shell_acc, 0, sizeof(unsigned long long) * pss::kShellWords * ns, c->stream));
    const double dV = c->dx[0] * c->dx[1] * (c->ndim == 3 ? c->dx[2] : 1.0);
    HIP_TRY(pss::launch_shells(c->stream, c->d_state[fd], c->n[0], c->n[1], c->ndim == 3 ? c->n[2] : 1, c->geo.tc,
                               c->mixed ? 1 : c->ndim, dV / static_cast<double>(c->sites()), ns, c->d_shell_acc));
    // shells 1 .. ns-1: the means, then the populations
    static_assert(sizeof(int64_t) == sizeof(unsigned long long), "count width");
    if (ns > 1) {
        HIP_TRY(hipMemcpyAsync(S, c->d_shell_acc + 1, sizeof(double) * (ns - 1), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipMemcpyAsync(counts, c->d_shell_acc + 2 * ns + 1, sizeof(int64_t) * (ns - 1), hipMemcpyDeviceToHost,
                               c->stream));
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    return PSS_OK;
}

pss_status pss_structure_factor_noalloc(pss_ctx* c, int32_t field, double* S, int64_t* counts, int32_t n_shells) {
    if (pss_status s = check_ctx(c)) return s;
    if (!S || !counts) return fail(PSS_E_INVAL, "null output");
    if (!c->planned) return fail(PSS_E_STATE, "the plan is not built (building it allocates device memory)");
    int fd = 0;
    if (pss_status s = dyn_field(c, field, &fd)) return s;
    if (pss_status s_bw = begin_work(c)) return s_bw;
    const int nmin = c->ndim == 3 ? std::min(std::min(c->n[0], c->n[1]), c->n[2])
                                  : (c->ndim == 2 ? std::min(c->n[0], c->n[1]) : c->n[0]);
    const int ns = nmin / 2;  // shells j = 1 .. ns-1
    if (n_shells != ns - 1) return fail(PSS_E_INVAL, "n_shells must be %d", ns - 1);
    if (ns > pss::kScratchShells)
        return fail(PSS_E_UNSUPPORTED, "%d shells exceed the %d of the static scratch", ns, pss::kScratchShells);
    void* base = nullptr;
    HIP_TRY(pss::scratch_address(&base));
    auto* acc = static_cast<unsigned long long*>(base);
    // the previous call's contents are still there: clear what is summed into
    HIP_TRY(pss::launch_zero_words(c->stream, acc, pss::kShellWords * ns));
    const double dV = c->dx[0] * c->dx[1] * (c->ndim == 3 ? c->dx[2] : 1.0);
    HIP_TRY(pss::launch_shells(c->stream, c->d_state[fd], c->n[0], c->n[1], c->ndim == 3 ? c->n[2] : 1, c->geo.tc,
                               c->mixed ? 1 : c->ndim, dV / static_cast<double>(c->sites()), ns, acc));
    // shells 1 .. ns-1 straight into the caller's arrays
    static_assert(sizeof(int64_t) == sizeof(unsigned long long), "count width");
    if (ns > 1) {
        HIP_TRY(hipMemcpyAsync(S, acc + 1, sizeof(double) * (ns - 1), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipMemcpyAsync(counts, acc + 2 * ns + 1, sizeof(int64_t) * (ns - 1), hipMemcpyDeviceToHost, c->stream));
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    return PSS_OK;
}

pss_status pss_util_philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                           int64_t count, uint32_t* out) {
    if (!out || count < 0) return fail(PSS_E_INVAL, "bad arguments");
    if (count == 0) return PSS_OK;
    HIP_TRY(pss::launch_philox(nullptr, c0, c1, c2, c3, k0, k1, count, out));
    HIP_TRY(hipStreamSynchronize(nullptr));
    return PSS_OK;
}

pss_status pss_kernels_per_step(pss_ctx* c, int32_t* count) {
    if (pss_status s = check_ctx(c)) return s;
    if (!count) return fail(PSS_E_INVAL, "null output");
    *count = c->ndim == 3 ? 4 : (c->ndim == 2 ? 2 : 1);
    return PSS_OK;
}

pss_status pss_kernel_bytes(pss_ctx* c, int32_t which, double* bytes) {
    if (pss_status s = check_ctx(c)) return s;
    if (!bytes) return fail(PSS_E_INVAL, "null output");
    if (pss_status s = materialize(c)) return s;
    const double arr = 8.0 * static_cast<double>(c->packed());  // one packed array
    const pss::DevPlan& P = c->plan;
    const int tc = c->geo.tc;
    const double lines = static_cast<double>(c->n[1]) * (c->ndim == 3 ? c->n[2] : 1);
    double vbytes = 0;  // factor arrays: only tiles holding kept columns move
    for (int g = 0; g < P.ng; ++g) {
        const int tiles = (P.mask[g].ncol + tc - 1) / tc;
        vbytes += 8.0 * tiles * tc * lines;
    }
    const int nf = static_cast<int>(c->fields.size());
    const int nk = c->ndim == 3 ? 4 : (c->ndim == 2 ? 2 : 1);
    if (which < 0 || which >= nk) return fail(PSS_E_INVAL, "kernel %d does not exist on this lattice", which);
    if (c->ndim == 1) {  // a one-step launch: every state in and out once
        *bytes = 2 * arr * nf;
        return PSS_OK;
    }
    if (c->mixed) {  // full arrays: channels in, state in/out, factors out; factors in, channels out
        *bytes = which == 0 ? arr * (P.nch + 2 * nf + P.ng) : arr * (P.ng + P.nch);
        return PSS_OK;
    }
    switch (which) {
        case 0: *bytes = arr * (P.nch + 2 * nf) + vbytes; break;  // channels in, state in/out, factors out
        case 1: *bytes = vbytes + arr * P.nch; break;             // factors in, channels out
        case 2: *bytes = 2 * vbytes; break;                       // factors in place
        default: *bytes = 2 * arr * P.nch; break;                 // channels re-laid out
    }
    return PSS_OK;
}

pss_status pss_time_kernel(pss_ctx* c, int32_t which, int32_t reps, double* ms, const char** name) {
    if (pss_status s = check_ctx(c)) return s;
    if (!ms || reps < 1) return fail(PSS_E_INVAL, "bad arguments");
    if (c->mixed) return fail(PSS_E_UNSUPPORTED, "kernel timing covers the power-of-two lattices");
    if (pss_status s = materialize(c)) return s;
    if (pss_status s_bw = begin_work(c)) return s_bw;
    const int nk = c->ndim == 3 ? 4 : (c->ndim == 2 ? 2 : 1);
    if (which < 0 || which >= nk) return fail(PSS_E_INVAL, "kernel %d does not exist on this lattice", which);
    // the x kernel and the y passes run only for models with real-space products
    if ((which == 1 || which == 3) && c->plan.nch == 0)
        return fail(PSS_E_INVAL, "kernel %d does not run on this model (no real-space products)", which);
    if (which == 2 && c->plan.ng == 0)
        return fail(PSS_E_INVAL, "kernel %d does not run on this model (no factor fields)", which);
    if (c->dirty)
        if (pss_status s = prologue(c)) return s;
    const int nf = static_cast<int>(c->fields.size());
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    pss::LaunchArgs a = args(c);
    const pss::LaunchArgs ax = xargs(c);
    HIP_TRY(hipEventRecord(e0, c->stream));
    a.nsteps = 1;  // 1D: one-step launches that leave the counter
    for (int r = 0; r < reps; ++r) {
        if (c->ndim == 1) {
            HIP_TRY(pss::launch_line1d(pss::MODE_STEP, c->n[0], nf, a));
            continue;
        }
        switch (which) {
            case 0: HIP_TRY(pss::launch_update(pss::MODE_STEP, c->lu, nf, a)); break;
            case 1: HIP_TRY(pss::launch_xrow(pss::MODE_STEP, c->n[0], c->plan.ng, ax)); break;
            case 2: HIP_TRY(y_inverse_factors(c)); break;
            default: HIP_TRY(y_forward_channels(c)); break;
        }
    }
    HIP_TRY(hipEventRecord(e1, c->stream));
    HIP_TRY(hipEventSynchronize(e1));
    float t = 0;
    HIP_TRY(hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = static_cast<double>(t) / reps;
    c->dirty = true;  // the channel arrays no longer match the state
    ++c->state_gen;   // repeated step launches changed the state
    static const char* names[4] = {"update_kernel", "xrow_kernel", "ypass_kernel(inverse)", "ypass_kernel(forward)"};
    if (name) *name = c->ndim == 1 ? "line1d_kernel" : names[which];
    return PSS_OK;
}

pss_status pss_autotune(pss_ctx* c, int32_t reps, double* us_per_step) {
    if (pss_status s = check_ctx(c)) return s;
    if (c->planned) return fail(PSS_E_STATE, "autotune before the plan is built (first upload, init or step)");
    if (reps < 1) return fail(PSS_E_INVAL, "reps must be >= 1");
    if (pss_status s = validate(c)) return s;
    if (c->ndim == 1 || c->mixed) {  // one block per line: no launch geometry to choose
        if (us_per_step) *us_per_step = 0.0;
        return PSS_OK;
    }
    using Tune = std::map<std::string, int64_t>;
    // one process-wide cache entry per device, lattice shape and term structure
    static std::map<std::string, std::pair<Tune, double>> cache;
    static std::mutex cache_mu;
    std::lock_guard<std::mutex> lock(cache_mu);
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    hipDeviceProp_t prop{};
    HIP_TRY(hipGetDeviceProperties(&prop, dev));
    std::string key = std::string("v1/") + prop.gcnArchName + "/" + std::to_string(c->ndim);
    for (int i = 0; i < c->ndim; ++i) key += "x" + std::to_string(c->n[i]);
    key += "/f" + std::to_string(c->fields.size()) + "/i" + std::to_string(c->interms.size()) + "/t";
    for (const Term& t : c->terms) {
        key += t.implicit ? "i" : "e";
        for (auto& fp : t.factors) key += std::to_string(fp.first) + "^" + std::to_string(fp.second);
        key += ",";
    }
    for (const auto& kv : c->tune) key += kv.first + "=" + std::to_string(kv.second);  // forced keys stay
    for (char& ch : key)
        if (std::isspace(static_cast<unsigned char>(ch))) ch = '_';
    // PSS_TUNE_CACHE names a text file that keeps the choices across
    // processes: one line per entry, "<key> <us per step> <k>=<v> ...", the
    // last line of a key wins; lines that do not parse are skipped
    const char* cache_file = std::getenv("PSS_TUNE_CACHE");
    if (cache_file && *cache_file && !cache.count(key)) {
        if (FILE* fp = std::fopen(cache_file, "r")) {
            char line[1024];
            while (std::fgets(line, sizeof line, fp)) {
                char* save = nullptr;
                const char* k = strtok_r(line, " \t\r\n", &save);
                const char* us = strtok_r(nullptr, " \t\r\n", &save);
                if (!k || !us || key != k) continue;
                char* end = nullptr;
                const double t = std::strtod(us, &end);
                if (*end || !(t > 0) || !std::isfinite(t)) continue;
                Tune tn;
                bool ok = true;
                while (const char* kv = strtok_r(nullptr, " \t\r\n", &save)) {
                    const char* eq = std::strchr(kv, '=');
                    const std::string name = eq ? std::string(kv, eq) : std::string();
                    const long long v = eq ? std::strtoll(eq + 1, &end, 10) : 0;
                    if (!eq || *end || v < 1 || v > 4096 ||
                        (name != "tc" && name != "to" && name != "tz" && name != "rb" && name != "pu" &&
                         name != "px" && name != "py")) {
                        ok = false;
                        break;
                    }
                    tn[name] = v;
                }
                if (ok) cache[key] = {tn, t};
            }
            std::fclose(fp);
        }
    }
    auto hit = cache.find(key);
    if (hit != cache.end()) {
        c->tune = hit->second.first;
        if (us_per_step) *us_per_step = hit->second.second;
        return PSS_OK;
    }
    // time the kernels of one step on a scratch copy of the model; +inf if
    // the geometry is not valid for this lattice
    const int nk = c->ndim == 3 ? 4 : 2;
    auto trial = [&](const Tune& tn) -> double {
        pss_ctx* t = new pss_ctx();
        t->ndim = c->ndim;
        for (int i = 0; i < 3; ++i) {
            t->n[i] = c->n[i];
            t->dx[i] = c->dx[i];
        }
        t->dt = c->dt;
        t->seed = c->seed;
        t->rule = c->rule;
        t->shape = c->shape;
        t->fields = c->fields;
        t->terms = c->terms;
        t->tune = tn;
        double total = 0;
        if (materialize(t) != PSS_OK) total = HUGE_VAL;
        for (int w = 0; w < nk && std::isfinite(total); ++w) {
            if ((w == 1 || w == 3) && t->plan.nch == 0) continue;
            if (w == 2 && t->plan.ng == 0) continue;
            double ms = 0;
            if (pss_time_kernel(t, w, reps, &ms, nullptr) != PSS_OK) {
                total = HUGE_VAL;
                break;
            }
            total += ms;
        }
        pss_lattice_destroy(t);
        return total;
    };
    const std::string err_keep = g_err;
    Tune best = c->tune;
    double tbest = trial(best);
    auto improve = [&](const char* k1, std::vector<int> v1, const char* k2, std::vector<int> v2) {
        const Tune base = best;
        // a key the caller set keeps its value
        if (c->tune.count(k1)) v1 = {static_cast<int>(c->tune.at(k1))};
        if (k2 && c->tune.count(k2)) v2 = {static_cast<int>(c->tune.at(k2))};
        for (int a : v1)
            for (int b : v2) {
                Tune tn = base;
                tn[k1] = a;
                if (k2) tn[k2] = b;
                const double tt = trial(tn);
                if (tt < tbest) {
                    tbest = tt;
                    best = tn;
                }
            }
    };
    // update kernel (and the tile width the x kernel shares), then x kernel,
    // then (3D) the y pass
    improve("pu", {4, 8, 16}, "tc", {1, 2, 4, 8, 16, 32});
    if (c->ndim == 3) improve("to", {1, 2, 4, 8}, nullptr, {0});
    improve("px", {4, 8, 16}, "rb", {2, 4, 8, 16, 32});
    if (c->ndim == 3) improve("py", {4, 8, 16}, "tz", {1, 2, 4, 8});
    g_err = err_keep;
    if (!std::isfinite(tbest)) return fail(PSS_E_UNSUPPORTED, "no launch geometry works for this lattice");
    c->tune = best;
    cache[key] = {best, tbest * 1e3};
    if (us_per_step) *us_per_step = tbest * 1e3;
    if (cache_file && *cache_file) {
        std::string line = key;
        char us[64];
        std::snprintf(us, sizeof us, " %.17g", tbest * 1e3);
        line += us;
        for (const auto& kv : best) line += " " + kv.first + "=" + std::to_string(kv.second);
        line += "\n";
        FILE* fp = std::fopen(cache_file, "a");
        const bool ok = fp && std::fwrite(line.data(), 1, line.size(), fp) == line.size();
        if (fp && std::fclose(fp) != 0) return fail(PSS_E_INVAL, "PSS_TUNE_CACHE: cannot write %s", cache_file);
        if (!ok) return fail(PSS_E_INVAL, "PSS_TUNE_CACHE: cannot append to %s", cache_file);
    }
    return PSS_OK;
}

pss_status pss_adjoint_model_b_forward(pss_ctx* c, int64_t nsteps, int32_t ckpt_every, const double* S_target,
                                       int32_t n_shells, double* loss, pss_tape** out) {
    if (!out) return fail(PSS_E_INVAL, "null tape output");
    *out = nullptr;
    if (pss_status s = check_ctx(c)) return s;
    if (nsteps < 1 || ckpt_every < 1) return fail(PSS_E_INVAL, "need nsteps >= 1 and ckpt_every >= 1");
    if (!S_target || !loss) return fail(PSS_E_INVAL, "null argument");
    if (c->ndim != 2 || c->mixed)
        return fail(PSS_E_UNSUPPORTED, "the adjoint is implemented for 2D lattices of power-of-two sizes");
    if (c->tapes > 0) return fail(PSS_E_STATE, "this lattice already holds an adjoint tape");
    // recognise Model B: one field; implicit -(a q^2 + k q^4); explicit -b q^2 F[phi^3]; noise D q^2
    double a = 0, b = 0, k = 0, D = 0;
    {
        bool ok = c->fields.size() == 1 && c->interms.empty() && c->terms.size() == 2 && !has_frames(c);
        int nimp = 0, ncub = 0;
        for (const Term& t : c->terms) {
            if (!ok) break;
            if (t.implicit) {
                ++nimp;
                for (const Mono& m : t.op) {
                    if (m.invq || m.iq[0] || m.iq[1] || m.iq[2] || (m.q2 != 1 && m.q2 != 2)) ok = false;
                    (m.q2 == 1 ? a : k) -= m.coef;
                }
            } else {
                ++ncub;
                ok = ok && t.factors.size() == 1 && t.factors[0].first == 0 && t.factors[0].second == 3 &&
                     t.op.size() == 1 && t.op[0].q2 == 1 && !t.op[0].invq && !t.op[0].iq[0] && !t.op[0].iq[1] &&
                     !t.op[0].iq[2];
                if (ok) b = -t.op[0].coef;
            }
        }
        const Field& f = c->fields.empty() ? Field{} : c->fields[0];
        if (f.noisy) {
            ok = ok && f.noise.size() == 1 && f.noise[0].q2 == 1 && !f.noise[0].invq && !f.noise[0].iq[0] &&
                 !f.noise[0].iq[1] && !f.noise[0].iq[2];
            if (ok) D = f.noise[0].coef;
        }
        if (!ok || nimp != 1 || ncub != 1)
            return fail(PSS_E_UNSUPPORTED, "the adjoint needs a Model B lattice (implicit a q^2 + k q^4, "
                                           "explicit -b q^2 phi^3, noise D q^2)");
    }
    if (pss_status s = materialize(c)) return s;
    if (pss_status s_bw = begin_work(c)) return s_bw;
    const int nx = c->n[0], ny = c->n[1];
    const int ns = std::min(nx, ny) / 2;
    if (n_shells != ns - 1) return fail(PSS_E_INVAL, "n_shells must be %d", ns - 1);

    auto* tp = new pss_tape();
    tp->ctx = c;
    tp->nsteps = nsteps;
    tp->ckpt = ckpt_every;
    tp->nck = (nsteps + ckpt_every - 1) / ckpt_every;
    tp->seglen = std::min<int64_t>(ckpt_every, nsteps);
    tp->fb = sizeof(float2) * static_cast<size_t>(c->packed());
    tp->ns = ns;
    tp->a = a;
    tp->b = b;
    tp->k = k;
    tp->D = D;
    auto bail = [&](pss_status st) {
        tape_free(tp);
        delete tp;
        return st;
    };
    // workspace: checkpoints, one recomputed segment, adjoint arrays
    const size_t fb = tp->fb;
    tp->ck = static_cast<char*>(tape_alloc(tp, fb * static_cast<size_t>(tp->nck)));
    tp->seg = static_cast<char*>(tape_alloc(tp, fb * static_cast<size_t>(tp->seglen + 1)));
    tp->fT = static_cast<float2*>(tape_alloc(tp, fb));
    tp->G = static_cast<float2*>(tape_alloc(tp, fb));
    tp->R0 = static_cast<float2*>(tape_alloc(tp, fb));
    tp->R1 = static_cast<float2*>(tape_alloc(tp, fb));
    tp->X = static_cast<float2*>(tape_alloc(tp, fb));
    tp->W = static_cast<float2*>(tape_alloc(tp, fb));
    tp->U = static_cast<float2*>(tape_alloc(tp, fb));
    tp->nacc = 3 * static_cast<size_t>(c->geo.nublk) + static_cast<size_t>(c->geo.nrowblk);
    tp->acc = static_cast<double*>(tape_alloc(tp, tp->nacc * sizeof(double)));
    tp->coef = static_cast<float*>(tape_alloc(tp, sizeof(float) * ns));
    tp->plan_row = static_cast<pss::DevPlan*>(tape_alloc(tp, sizeof(pss::DevPlan)));
    tp->plan_raw = static_cast<pss::DevPlan*>(tape_alloc(tp, sizeof(pss::DevPlan)));
    if (tp->mem.size() != 13)
        return bail(fail(PSS_E_NOMEM, "adjoint workspace of %zu bytes does not fit",
                         fb * static_cast<size_t>(tp->nck + tp->seglen + 8)));
#define TAPE_HIP(expr)                                                                                      \
    do {                                                                                                    \
        hipError_t e_ = (expr);                                                                             \
        if (e_ != hipSuccess)                                                                               \
            return bail(fail(PSS_E_HIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__)); \
    } while (0)
#define TAPE_TRY(expr)          \
    do {                        \
        pss_status s_ = (expr); \
        if (s_) return bail(s_); \
    } while (0)

    // plans of the row pass (u from the kept columns, w from all) and of the
    // unnormalised inverse transform of g_0
    pss::DevPlan pr = c->plan;
    pr.mask[1] = pr.mask[0];
    pr.mask[1].ncol = nx / 2;
    pr.ng = 2;
    pss::DevPlan pu = c->plan;
    pu.inv_n = 1.f;
    TAPE_HIP(hipMemcpy(tp->plan_row, &pr, sizeof(pr), hipMemcpyHostToDevice));
    TAPE_HIP(hipMemcpy(tp->plan_raw, &pu, sizeof(pu), hipMemcpyHostToDevice));

    // forward run with a checkpoint every ckpt_every steps
    tp->n0 = c->steps_taken;
    for (int64_t sgi = 0; sgi < tp->nck; ++sgi) {
        if (c->dirty) TAPE_TRY(prologue(c));
        TAPE_HIP(hipMemcpyAsync(tape_at(tp, tp->ck, sgi), c->d_state[0], fb, hipMemcpyDeviceToDevice, c->stream));
        TAPE_TRY(pss_step(c, std::min<int64_t>(ckpt_every, nsteps - sgi * ckpt_every)));
    }
    TAPE_HIP(hipMemcpyAsync(tp->fT, c->d_state[0], fb, hipMemcpyDeviceToDevice, c->stream));

    // loss and terminal seed from the shell averages of the final spectrum
    std::vector<double> S(ns - 1);
    std::vector<int64_t> cnt(ns - 1);
    TAPE_TRY(pss_structure_factor(c, 0, S.data(), cnt.data(), ns - 1));
    const double dV = c->dx[0] * c->dx[1];
    const double N = static_cast<double>(c->sites());
    double L = 0;
    std::vector<float> cf(ns, 0.f);
    for (int j = 1; j < ns; ++j) {
        const double d = S[j - 1] - S_target[j - 1];
        L += d * d;
        cf[j] = static_cast<float>(2.0 * d / std::max<int64_t>(cnt[j - 1], 1) * (dV / N) * 2.0);
    }
    TAPE_HIP(hipMemcpy(tp->coef, cf.data(), sizeof(float) * ns, hipMemcpyHostToDevice));
#undef TAPE_HIP
#undef TAPE_TRY
    tp->loss = L;
    tp->plan_gen = c->plan_gen;
    tp->state_gen = c->state_gen;
    ++c->tapes;
    *loss = L;
    *out = tp;
    return PSS_OK;
}

pss_status pss_adjoint_model_b_backward(pss_tape* tp, double* grad, float* grad_phi0, int32_t on_device) {
    if (!tp) return fail(PSS_E_INVAL, "null tape");
    if (!grad) return fail(PSS_E_INVAL, "null gradient output");
    if (tp->done) return fail(PSS_E_STATE, "the reverse sweep of this tape has already run");
    pss_ctx* c = tp->ctx;
    if (c->plan_gen != tp->plan_gen || c->state_gen != tp->state_gen)
        return fail(PSS_E_STATE, "the lattice changed (coefficients, seed or state) after the forward run");
    if (pss_status s = begin_work(c)) return s;
    const int nx = c->n[0], ny = c->n[1];
    const size_t fb = tp->fb;
#define ADJ_HIP(expr)                                                                                \
    do {                                                                                             \
        hipError_t e_ = (expr);                                                                      \
        if (e_ != hipSuccess)                                                                        \
            return fail(PSS_E_HIP, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, __LINE__); \
    } while (0)
    tp->done = true;
    ADJ_HIP(pss::launch_adjseed(c->stream, tp->fT, tp->G, tp->coef, tp->ns, nx, ny, c->geo.tc));
    ADJ_HIP(hipMemsetAsync(tp->acc, 0, tp->nacc * sizeof(double), c->stream));

    // reverse sweep: recompute each segment from its checkpoint, then step back
    pss::AdjArgs aa{};
    aa.plan = c->d_plan;
    aa.G = tp->G;
    aa.X = tp->X;
    aa.W = tp->W;
    aa.U = tp->U;
    aa.acc = tp->acc;
    aa.a = static_cast<float>(tp->a);
    aa.b = static_cast<float>(tp->b);
    aa.k = static_cast<float>(tp->k);
    aa.D = static_cast<float>(tp->D);
    aa.first = 1;
    float2* Rcur = tp->R0;
    float2* Rnxt = tp->R1;
    pss::LaunchArgs ax = args(c);
    ax.plan = tp->plan_row;
    ax.bufs = pss::Bufs{};
    ax.bufs.V[0] = tp->U;
    ax.bufs.V[1] = tp->W;
    ax.bufs.N[0] = tp->X;
    ax.bufs.acc = tp->acc + 3 * static_cast<size_t>(c->geo.nublk);
    const int64_t n0 = tp->n0, nsteps = tp->nsteps;
    for (int64_t sgi = tp->nck - 1; sgi >= 0; --sgi) {
        const int64_t start = sgi * tp->ckpt;
        const int64_t len = std::min<int64_t>(tp->ckpt, nsteps - start);
        const uint64_t st = static_cast<uint64_t>(n0 + start);
        ADJ_HIP(hipStreamSynchronize(c->stream));
        ADJ_HIP(hipMemcpy(c->d_step, &st, sizeof(st), hipMemcpyHostToDevice));
        ADJ_HIP(hipMemcpyAsync(c->d_state[0], tape_at(tp, tp->ck, sgi), fb, hipMemcpyDeviceToDevice, c->stream));
        ADJ_HIP(hipMemcpyAsync(tape_at(tp, tp->seg, 0), tape_at(tp, tp->ck, sgi), fb, hipMemcpyDeviceToDevice,
                               c->stream));
        if (pss_status s = prologue(c)) return s;
        for (int64_t i = 1; i <= len; ++i) {
            if (pss_status s = enqueue_steps(c, 1)) return s;
            ADJ_HIP(hipMemcpyAsync(tape_at(tp, tp->seg, i), c->d_state[0], fb, hipMemcpyDeviceToDevice, c->stream));
        }
        for (int64_t i = len - 1; i >= 0; --i) {
            aa.Rin = Rcur;
            aa.Rout = Rnxt;
            aa.phi1 = tape_at(tp, tp->seg, i + 1);
            aa.phi0 = tape_at(tp, tp->seg, i);
            aa.step = static_cast<uint32_t>(n0 + start + i);
            ADJ_HIP(pss::launch_adjcol(pss::MODE_ADJCOL, ny, aa, args(c)));
            ADJ_HIP(pss::launch_xrow(pss::MODE_ADJROW, nx, 2, ax));
            std::swap(Rcur, Rnxt);
            aa.first = 0;
        }
    }
    // g_0, and the gradient for the real initial field: N F^-1[g_0]
    aa.Rin = Rcur;
    aa.Rout = tp->G;
    ADJ_HIP(pss::launch_adjcol(pss::MODE_ADJFIN, ny, aa, args(c)));
    std::vector<double> slots(tp->nacc);
    ADJ_HIP(hipMemcpyAsync(slots.data(), tp->acc, tp->nacc * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    if (grad_phi0) {
        pss::LaunchArgs a1 = args(c);
        a1.plan = tp->plan_raw;
        a1.bufs.S[0] = tp->G;
        a1.bufs.sel = 0;
        a1.bufs.out = c->d_tmp;
        ADJ_HIP(pss::launch_update(pss::MODE_INV_OUT, c->lu, 1, a1));
        a1.bufs.in = c->d_tmp;
        a1.bufs.real_out = c->d_real;
        ADJ_HIP(pss::launch_xrow(pss::MODE_C2R_OUT, nx, 1, a1));
        ADJ_HIP(hipMemcpyAsync(grad_phi0, c->d_real, sizeof(float) * static_cast<size_t>(c->sites()),
                               on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
    }
    // leave the lattice at the end of the forward run
    const uint64_t fin = static_cast<uint64_t>(n0 + nsteps);
    ADJ_HIP(hipStreamSynchronize(c->stream));
    ADJ_HIP(hipMemcpy(c->d_step, &fin, sizeof(fin), hipMemcpyHostToDevice));
    ADJ_HIP(hipMemcpy(c->d_state[0], tp->fT, fb, hipMemcpyDeviceToDevice));
#undef ADJ_HIP
    c->steps_taken = n0 + nsteps;
    c->dirty = true;
    ++c->state_gen;
    // the per-block slots in block order: dL/da, dL/dk, dL/dD from the
    // column blocks, dL/db from the row blocks
    double gh[4] = {0.0, 0.0, 0.0, 0.0};
    const size_t ncol = static_cast<size_t>(c->geo.nublk);
    for (size_t bk = 0; bk < ncol; ++bk) {
        gh[0] += slots[3 * bk];
        gh[2] += slots[3 * bk + 1];
        gh[3] += slots[3 * bk + 2];
    }
    for (size_t bk = 3 * ncol; bk < tp->nacc; ++bk) gh[1] += slots[bk];
    for (int i = 0; i < 4; ++i) grad[i] = gh[i];
    return PSS_OK;
}

pss_status pss_tape_destroy(pss_tape* tp) {
    if (!tp) return PSS_OK;
    tape_free(tp);
    --tp->ctx->tapes;
    delete tp;
    return PSS_OK;
}

pss_status pss_adjoint_model_b(pss_ctx* c, int64_t nsteps, int32_t ckpt_every, const double* S_target,
                               int32_t n_shells, double* loss, double* grad, float* grad_phi0, int32_t on_device) {
    if (!grad) return fail(PSS_E_INVAL, "null argument");
    pss_tape* tp = nullptr;
    if (pss_status s = pss_adjoint_model_b_forward(c, nsteps, ckpt_every, S_target, n_shells, loss, &tp)) return s;
    const pss_status s = pss_adjoint_model_b_backward(tp, grad, grad_phi0, on_device);
    pss_tape_destroy(tp);
    return s;
}

pss_status pss_batch_create(pss_batch** out, pss_ctx* const* lattices, int32_t n, const uint64_t* seeds) {
    if (!out) return fail(PSS_E_INVAL, "null output");
    *out = nullptr;
    if (!lattices || n < 1) return fail(PSS_E_INVAL, "a batch needs at least one lattice");
    for (int32_t i = 0; i < n; ++i) {
        if (!lattices[i]) return fail(PSS_E_INVAL, "lattice %d is null", i);
        if (lattices[i]->ndim != 2 || lattices[i]->mixed)
            return fail(PSS_E_UNSUPPORTED, "lattice %d: batches hold 2D lattices of power-of-two sizes only", i);
        if (has_frames(lattices[i]))
            return fail(PSS_E_UNSUPPORTED, "lattice %d has boundary frames, which batched steps do not apply", i);
        for (int32_t j = 0; j < i; ++j)
            if (lattices[j] == lattices[i]) return fail(PSS_E_INVAL, "lattice %d appears twice", i);
    }
    for (int32_t i = 0; i < n; ++i) {
        if (seeds)
            if (pss_status s = pss_seed_set(lattices[i], seeds[i])) return s;
        if (pss_status s = materialize(lattices[i])) return s;
    }
    auto* b = new pss_batch();
    b->mem.assign(lattices, lattices + n);
    b->seen.assign(n, ~uint64_t{0});
    for (int32_t i = 0; i < n; ++i) b->all.push_back(i);
    for (int32_t i = 0; i < n; ++i) {
        auto it = std::find_if(b->cls.begin(), b->cls.end(),
                               [&](const pss_batch::Class& cl) { return same_class(cl.rep, lattices[i]); });
        if (it == b->cls.end()) {
            b->cls.emplace_back();
            b->cls.back().rep = lattices[i];
            it = b->cls.end() - 1;
        }
        it->idx.push_back(i);
    }
    auto bail = [&](pss_status s) {
        free_batch(b);
        delete b;
        return s;
    };
    std::vector<uint64_t*> ctrs;
    for (pss_ctx* c : b->mem) ctrs.push_back(c->d_step);
    hipError_t e = hipMalloc(&b->d_ctrs, sizeof(uint64_t*) * ctrs.size());
    if (e == hipSuccess) e = hipMalloc(&b->d_flags, sizeof(uint32_t) * ctrs.size());
    if (e == hipSuccess) e = hipMemcpy(b->d_ctrs, ctrs.data(), sizeof(uint64_t*) * ctrs.size(), hipMemcpyHostToDevice);
    for (auto& cl : b->cls) {
        std::vector<pss::Member> tu, tx;
        for (int i : cl.idx) {
            tu.push_back(member_u(b->mem[i]));
            tx.push_back(member_x(b->mem[i]));
        }
        const size_t bytes = sizeof(pss::Member) * tu.size();
        if (e == hipSuccess) e = hipMalloc(&cl.d_u, bytes);
        if (e == hipSuccess) e = hipMalloc(&cl.d_x, bytes);
        if (e == hipSuccess) e = hipMalloc(&cl.d_plans, sizeof(pss::DevPlan) * tu.size());
        if (e == hipSuccess) e = hipMemcpy(cl.d_u, tu.data(), bytes, hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemcpy(cl.d_x, tx.data(), bytes, hipMemcpyHostToDevice);
        for (size_t j = 0; j < cl.idx.size() && e == hipSuccess; ++j) {
            pss_ctx* m = b->mem[cl.idx[j]];
            e = hipMemcpy(cl.d_plans + j, m->d_plan, sizeof(pss::DevPlan), hipMemcpyDeviceToDevice);
            cl.gen.push_back(m->plan_gen);
        }
    }
    if (e == hipSuccess) e = hipEventCreateWithFlags(&b->ev, hipEventDisableTiming);
    if (e != hipSuccess)
        return bail(fail(e == hipErrorOutOfMemory ? PSS_E_NOMEM : PSS_E_HIP, "batch set-up: %s", hipGetErrorString(e)));
    b->stream = b->mem[0]->stream;
    const char* env = std::getenv("PSS_BATCH_RESIDENT");
    b->resident = !(env && std::strcmp(env, "0") == 0);
    batch_plan_fused(b);
    for (pss_ctx* c : b->mem) ++c->batches;
    *out = b;
    return PSS_OK;
}

pss_status pss_batch_destroy(pss_batch* b) {
    if (!b) return PSS_OK;
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    for (pss_ctx* c : b->mem) {
        --c->batches;
        if (c->after_batch == b->ev) c->after_batch = nullptr;  // its work is done
    }
    free_batch(b);
    delete b;
    return PSS_OK;
}

pss_status pss_batch_step(pss_batch* b, int64_t nsteps) {
    if (!b) return fail(PSS_E_INVAL, "null batch");
    if (nsteps < 0) return fail(PSS_E_INVAL, "negative step count");
    if (nsteps == 0) return PSS_OK;
    // channel arrays of every member must match its state; the batch stream
    // comes after every member's own work
    if (pss_status s = batch_order_before(b, b->all)) return s;
    if (pss_status s = batch_refresh_plans(b)) return s;
    int64_t left = nsteps;
    while (left > 0) {
        const int64_t k = std::min(left, kGraphSteps);
        hipGraphExec_t ex = nullptr;
        if (pss_status s = batch_graph_for(b, k, &ex)) return s;
        HIP_TRY(hipGraphLaunch(ex, b->stream));
        left -= k;
    }
    // later work on any member's stream comes after the batch
    if (pss_status s = batch_order_after(b, b->all)) return s;
    for (pss_ctx* c : b->mem) {
        c->steps_taken += nsteps;
        ++c->state_gen;
    }
    return PSS_OK;
}

pss_status pss_batch_sync(pss_batch* b) {
    if (!b) return fail(PSS_E_INVAL, "null batch");
    HIP_TRY(hipStreamSynchronize(b->stream));
    // every member's flag read and cleared by one kernel and one copy
    const int n = static_cast<int>(b->mem.size());
    std::vector<uint32_t> flags(n);
    HIP_TRY(pss::launch_take_flags(b->stream, b->d_ctrs, n, b->d_flags));
    HIP_TRY(hipMemcpyAsync(flags.data(), b->d_flags, sizeof(uint32_t) * n, hipMemcpyDeviceToHost, b->stream));
    HIP_TRY(hipStreamSynchronize(b->stream));
    for (int i = 0; i < n; ++i)
        if (flags[i])  // report the first member; every flag is cleared
            return fail(PSS_E_NONFINITE,
                        "member %d: a non-finite value appeared in the state (field mask 0x%x) at or before step %lld",
                        i, flags[i], static_cast<long long>(b->mem[i]->steps_taken));
    return PSS_OK;
}

pss_status pss_batch_launches(pss_batch* b, int32_t* per_step, int32_t* fused_classes, int32_t* resident_classes) {
    if (!b) return fail(PSS_E_INVAL, "null batch");
    if (per_step) *per_step = batch_launches_per_step(b);
    if (fused_classes) *fused_classes = b->fu.ncls;
    if (resident_classes) *resident_classes = static_cast<int32_t>(b->res.size());
    return PSS_OK;
}

pss_status pss_batch_info(pss_batch* b, int32_t* n_classes, int32_t* class_of) {
    if (!b) return fail(PSS_E_INVAL, "null batch");
    if (n_classes) *n_classes = static_cast<int32_t>(b->cls.size());
    if (class_of)
        for (size_t k = 0; k < b->cls.size(); ++k)
            for (int i : b->cls[k].idx) class_of[i] = static_cast<int32_t>(k);
    return PSS_OK;
}

pss_status pss_batch_time_kernel(pss_batch* b, int32_t cls, int32_t which, int32_t reps, double* ms,
                                 double* bytes) {
    if (!b) return fail(PSS_E_INVAL, "null batch");
    if ((which != 0 && which != 1) || reps < 1 || !ms) return fail(PSS_E_INVAL, "bad kernel timing request");
    if (cls == -1) return batch_time_fused(b, which, reps, ms, bytes);
    if (cls == -2) return batch_time_resident(b, reps, ms, bytes);
    if (cls < 0 || cls >= static_cast<int32_t>(b->cls.size())) return fail(PSS_E_INVAL, "no class %d", cls);
    const auto& cl = b->cls[cls];
    pss_ctx* r = cl.rep;
    if (which == 1 && r->plan.nch == 0) return fail(PSS_E_INVAL, "class %d has no x kernel", cls);
    if (pss_status s = batch_order_before(b, cl.idx)) return s;
    if (pss_status s = batch_refresh_plans(b)) return s;
    pss::LaunchArgs a = which == 0 ? args(r) : xargs(r);
    a.stream = b->stream;
    a.members = which == 0 ? cl.d_u : cl.d_x;
    a.plans = cl.d_plans;
    a.nmem = static_cast<int>(cl.idx.size());
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    HIP_TRY(hipEventRecord(e0, b->stream));
    for (int k = 0; k < reps; ++k) {
        if (which == 0)
            HIP_TRY(pss::launch_update(pss::MODE_STEP, r->lu, static_cast<int>(r->fields.size()), a));
        else
            HIP_TRY(pss::launch_xrow(pss::MODE_STEP, r->n[0], r->plan.ng, a));
    }
    HIP_TRY(hipEventRecord(e1, b->stream));
    HIP_TRY(hipEventSynchronize(e1));
    float t = 0;
    HIP_TRY(hipEventElapsedTime(&t, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    *ms = static_cast<double>(t) / reps;
    if (bytes) {
        double one = 0;
        if (pss_status s = pss_kernel_bytes(r, which, &one)) return s;
        *bytes = one * static_cast<double>(cl.idx.size());
    }
    for (int i : cl.idx) {  // repeated launches leave the channels stale and change the states
        b->mem[i]->dirty = true;
        ++b->mem[i]->state_gen;
    }
    if (pss_status s = batch_order_after(b, cl.idx)) return s;
    return PSS_OK;
}

}  // extern "C"
