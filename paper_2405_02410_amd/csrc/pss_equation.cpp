// Equation-string front end (Sec. "Writing models" and its "Reserved
// keywords" subsection): parses the paper's equation strings into calls of
// the C interface (pss_term_add, pss_noise_set).  It holds no numerics of the
// method: an equation becomes a polynomial in the fields whose coefficients
// are q-operator monomials, and each group of monomials with the same field
// factors becomes one term.
//
// Grammar (whitespace ignored):
//   equation := ["dt"] NAME [("+" | "-") sum] "=" (sum | "0")
//   sum      := ["+" | "-"] term {("+" | "-") term}
//   term     := power {("*" power) | ("/" divisor)}
//   divisor  := NUMBER | PARAM | "q" ["^" INT]           (1/q: |q|^-1)
//   power    := atom ["^" INT]
//   atom     := NUMBER | PARAM | FIELD | "q" "^" EVEN | "iqx" | "iqy" | "iqz"
//             | "(" sum ")"
// "dt phi" marks the equation of dynamic field phi; an equation without "dt"
// defines an intermediate field.  The left-hand side after the field must be
// linear in that field (implicit terms, moved to the right-hand side with
// their sign flipped); the right-hand side may hold any products of fields.
// q^(2n) is (q^2)^n, i.e. (-laplacian)^n; iqx, iqy, iqz are the derivatives;
// "/q" divides by |q|.
#include <algorithm>
#include <cctype>
#include <cstdarg>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <map>
#include <string>
#include <utility>
#include <vector>

#include "../../include/pss.h"
#include "pss_error.h"

namespace {

pss_status fail(pss_status code, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    const pss_status s = pss_internal::set_error(code, fmt, ap);
    va_end(ap);
    return s;
}

// one product of operator powers and field powers
struct Key {
    int q2 = 0, invq = 0, iq[3] = {0, 0, 0};
    std::vector<std::pair<int, int>> fields;  // (field id, power), sorted by id
    bool operator<(const Key& o) const {
        if (q2 != o.q2) return q2 < o.q2;
        if (invq != o.invq) return invq < o.invq;
        for (int i = 0; i < 3; ++i)
            if (iq[i] != o.iq[i]) return iq[i] < o.iq[i];
        return fields < o.fields;
    }
};
using Poly = std::map<Key, double>;

Poly constant(double v) {
    Poly p;
    p[Key{}] = v;
    return p;
}

Poly product(const Poly& a, const Poly& b) {
    Poly r;
    for (const auto& x : a)
        for (const auto& y : b) {
            Key k = x.first;
            k.q2 += y.first.q2;
            k.invq += y.first.invq;
            for (int i = 0; i < 3; ++i) k.iq[i] += y.first.iq[i];
            for (const auto& fp : y.first.fields) {
                bool found = false;
                for (auto& kf : k.fields)
                    if (kf.first == fp.first) {
                        kf.second += fp.second;
                        found = true;
                    }
                if (!found) k.fields.push_back(fp);
            }
            std::sort(k.fields.begin(), k.fields.end());
            r[k] += x.second * y.second;
        }
    return r;
}

void add_to(Poly& a, const Poly& b, double sign) {
    for (const auto& x : b) a[x.first] += sign * x.second;
}

class Parser {
public:
    Parser(pss_ctx* ctx, const char* text) : ctx_(ctx), s_(text) {}

    pss_status error() const { return err_; }
    size_t pos() const { return i_; }

    void skip() {
        while (s_[i_] && std::isspace(static_cast<unsigned char>(s_[i_]))) ++i_;
    }
    bool at_end() {
        skip();
        return s_[i_] == 0;
    }
    char peek() {
        skip();
        return s_[i_];
    }
    bool accept(char ch) {
        if (peek() != ch) return false;
        ++i_;
        return true;
    }
    bool ident(std::string* out) {
        skip();
        const size_t b = i_;
        if (!(std::isalpha(static_cast<unsigned char>(s_[i_])) || s_[i_] == '_')) return false;
        while (std::isalnum(static_cast<unsigned char>(s_[i_])) || s_[i_] == '_') ++i_;
        *out = std::string(s_ + b, i_ - b);
        return true;
    }
    bool number(double* v) {
        skip();
        if (!(std::isdigit(static_cast<unsigned char>(s_[i_])) || s_[i_] == '.')) return false;
        char* end = nullptr;
        *v = std::strtod(s_ + i_, &end);
        if (end == s_ + i_) return false;
        i_ = static_cast<size_t>(end - s_);
        return true;
    }
    bool integer(int* v) {
        skip();
        const bool neg = s_[i_] == '-';
        const size_t b = i_ + (neg ? 1 : 0);
        if (!std::isdigit(static_cast<unsigned char>(s_[b]))) return false;
        size_t e = b;
        long n = 0;
        while (std::isdigit(static_cast<unsigned char>(s_[e]))) n = 10 * n + (s_[e++] - '0');
        i_ = e;
        *v = static_cast<int>(neg ? -n : n);
        return true;
    }
    void set_error(pss_status st, const char* what) {
        if (err_ == PSS_OK) err_ = fail(st, "equation, at character %zu: %s", i_, what);
    }

    Poly sum() {
        Poly r;
        double sign = 1.0;
        if (accept('-'))
            sign = -1.0;
        else
            accept('+');
        add_to(r, term(), sign);
        while (err_ == PSS_OK) {
            if (accept('+'))
                add_to(r, term(), 1.0);
            else if (accept('-'))
                add_to(r, term(), -1.0);
            else
                break;
        }
        return r;
    }

    Poly term() {
        Poly r = power();
        while (err_ == PSS_OK) {
            if (accept('*')) {
                r = product(r, power());
            } else if (accept('/')) {
                r = product(r, divisor());
            } else {
                break;
            }
        }
        return r;
    }

    Poly divisor() {
        double v;
        if (number(&v)) {
            if (v == 0) set_error(PSS_E_INVAL, "division by zero");
            return constant(v == 0 ? 0.0 : 1.0 / v);
        }
        std::string id;
        if (!ident(&id)) {
            set_error(PSS_E_INVAL, "expected a number, a parameter or q after '/'");
            return constant(0);
        }
        if (id == "q") {
            int n = 1;
            if (accept('^') && (!integer(&n) || n < 1)) set_error(PSS_E_INVAL, "1/q takes a positive power");
            Key k;
            k.invq = n;
            Poly p;
            p[k] = 1.0;
            return p;
        }
        double pv;
        if (pss_param_get(ctx_, id.c_str(), &pv) == PSS_OK) {
            if (pv == 0) set_error(PSS_E_INVAL, "division by a zero parameter");
            return constant(pv == 0 ? 0.0 : 1.0 / pv);
        }
        set_error(PSS_E_INVAL, "only numbers, parameters and q can divide");
        return constant(0);
    }

    Poly power() {
        Poly base = atom();
        if (err_ == PSS_OK && !q_power_done_ && accept('^')) {
            int n = 0;
            if (!integer(&n) || n < 0) {
                set_error(PSS_E_INVAL, "a power must be a non-negative integer");
                return base;
            }
            Poly r = constant(1.0);
            for (int k = 0; k < n; ++k) r = product(r, base);
            return r;
        }
        q_power_done_ = false;
        return base;
    }

    Poly atom() {
        q_power_done_ = false;
        double v;
        if (accept('(')) {
            Poly r = sum();
            if (!accept(')')) set_error(PSS_E_INVAL, "missing ')'");
            return r;
        }
        if (number(&v)) return constant(v);
        std::string id;
        if (!ident(&id)) {
            set_error(PSS_E_INVAL, "expected a number, a name or '('");
            return constant(0);
        }
        if (id == "dt") {
            set_error(PSS_E_INVAL, "'dt' may only open an equation");
            return constant(0);
        }
        if (id == "q") {
            // q carries an even power: q^(2n) = (q^2)^n
            int n = 0;
            if (!accept('^') || !integer(&n) || n < 0 || (n & 1)) {
                set_error(PSS_E_INVAL, "q must carry an even power (q^2, q^4, ...)");
                return constant(0);
            }
            q_power_done_ = true;
            Key k;
            k.q2 = n / 2;
            Poly p;
            p[k] = 1.0;
            return p;
        }
        if (id == "iqx" || id == "iqy" || id == "iqz") {
            Key k;
            k.iq[id[2] - 'x'] = 1;
            Poly p;
            p[k] = 1.0;
            return p;
        }
        int32_t fid = 0, dyn = 0;
        if (pss_field_find(ctx_, id.c_str(), &fid, &dyn) == PSS_OK) {
            Key k;
            k.fields.push_back({fid, 1});
            Poly p;
            p[k] = 1.0;
            return p;
        }
        double pv;
        if (pss_param_get(ctx_, id.c_str(), &pv) == PSS_OK) return constant(pv);
        std::string msg = "unknown name '" + id + "' (not a field, a parameter or a keyword)";
        set_error(PSS_E_INVAL, msg.c_str());
        return constant(0);
    }

private:
    pss_ctx* ctx_;
    const char* s_;
    size_t i_ = 0;
    pss_status err_ = PSS_OK;
    bool q_power_done_ = false;
};

// the monomials of one operator (keys with the same fields) as pss_qmono
void to_monos(const std::vector<std::pair<Key, double>>& terms, std::vector<pss_qmono>* out) {
    for (const auto& t : terms) {
        pss_qmono m{};
        m.coef = t.second;
        m.q2_pow = t.first.q2;
        m.invq_pow = t.first.invq;
        for (int i = 0; i < 3; ++i) m.iq_pow[i] = t.first.iq[i];
        out->push_back(m);
    }
}

// add the monomials as terms of `target` (at most 8 monomials a term)
pss_status add_terms(pss_ctx* ctx, int32_t target, int32_t implicit, const std::vector<pss_qmono>& ops,
                     const std::vector<std::pair<int, int>>& fields, int32_t* first, int32_t* count) {
    std::vector<int32_t> ff, fp;
    for (const auto& f : fields) {
        ff.push_back(f.first);
        fp.push_back(f.second);
    }
    for (size_t b = 0; b < ops.size(); b += 8) {
        const int32_t nm = static_cast<int32_t>(std::min<size_t>(8, ops.size() - b));
        int32_t id = -1;
        if (pss_status s = pss_term_add(ctx, target, implicit, ops.data() + b, nm, ff.data(), fp.data(),
                                        static_cast<int32_t>(ff.size()), &id))
            return s;
        if (*count == 0) *first = id;
        ++*count;
    }
    return PSS_OK;
}

}  // namespace

extern "C" pss_status pss_equation_add(pss_ctx* ctx, const char* equation, int32_t* first_term, int32_t* n_terms) {
    if (!ctx || !equation) return fail(PSS_E_INVAL, "null argument");
    Parser ps(ctx, equation);
    // "dt NAME" or "NAME"
    std::string name;
    if (!ps.ident(&name)) return fail(PSS_E_INVAL, "an equation opens with 'dt <field>' or '<field>'");
    bool dt = false;
    if (name == "dt") {
        dt = true;
        if (!ps.ident(&name)) return fail(PSS_E_INVAL, "'dt' must be followed by a field name");
    }
    int32_t target = 0, dynamic = 0;
    if (pss_status s = pss_field_find(ctx, name.c_str(), &target, &dynamic)) return s;
    if (dt != (dynamic != 0))
        return fail(PSS_E_INVAL, dt ? "'%s' is an intermediate field: its equation has no 'dt'"
                                    : "'%s' is a dynamic field: its equation opens with 'dt'",
                    name.c_str());
    Poly lhs;
    if (ps.peek() != '=') {
        const char c = ps.peek();
        if (c != '+' && c != '-') return fail(PSS_E_INVAL, "expected '+', '-' or '=' after '%s'", name.c_str());
        lhs = ps.sum();
        if (ps.error()) return ps.error();
    }
    if (!ps.accept('=')) return fail(PSS_E_INVAL, "expected '=' at character %zu", ps.pos());
    Poly rhs = ps.sum();
    if (ps.error()) return ps.error();
    if (!ps.at_end()) return fail(PSS_E_INVAL, "unexpected text at character %zu", ps.pos());

    // implicit terms: linear in the target, moved to the right-hand side
    std::vector<std::pair<Key, double>> imp;
    for (const auto& t : lhs) {
        if (t.second == 0.0) continue;
        if (!(t.first.fields.size() == 1 && t.first.fields[0].first == target && t.first.fields[0].second == 1))
            return fail(PSS_E_INVAL, "every left-hand-side term must be linear in '%s' (implicit terms)",
                        name.c_str());
        Key op = t.first;
        op.fields.clear();
        imp.push_back({op, -t.second});
    }
    // explicit terms grouped by their field factors
    std::map<std::vector<std::pair<int, int>>, std::vector<std::pair<Key, double>>> groups;
    for (const auto& t : rhs) {
        if (t.second == 0.0) continue;
        if (t.first.fields.empty())
            return fail(PSS_E_UNSUPPORTED, "a right-hand-side term without fields (a source) is not supported");
        Key op = t.first;
        op.fields.clear();
        groups[t.first.fields].push_back({op, t.second});
    }
    int32_t first = -1, count = 0;
    if (!imp.empty()) {
        std::vector<pss_qmono> ops;
        to_monos(imp, &ops);
        if (pss_status s = add_terms(ctx, target, 1, ops, {{target, 1}}, &first, &count)) return s;
    }
    for (const auto& g : groups) {
        std::vector<pss_qmono> ops;
        to_monos(g.second, &ops);
        if (pss_status s = add_terms(ctx, target, 0, ops, g.first, &first, &count)) return s;
    }
    if (first_term) *first_term = first;
    if (n_terms) *n_terms = count;
    return PSS_OK;
}

extern "C" pss_status pss_noise_expr(pss_ctx* ctx, int32_t field, const char* expr) {
    if (!ctx || !expr) return fail(PSS_E_INVAL, "null argument");
    Parser ps(ctx, expr);
    Poly p = ps.sum();
    if (ps.error()) return ps.error();
    if (!ps.at_end()) return fail(PSS_E_INVAL, "unexpected text at character %zu", ps.pos());
    std::vector<std::pair<Key, double>> mono;
    for (const auto& t : p) {
        if (t.second == 0.0) continue;
        if (!t.first.fields.empty()) return fail(PSS_E_INVAL, "a noise prefactor holds no fields");
        mono.push_back(t);
    }
    if (mono.empty()) return fail(PSS_E_INVAL, "the noise prefactor is zero");
    std::vector<pss_qmono> ops;
    to_monos(mono, &ops);
    return pss_noise_set(ctx, field, ops.data(), static_cast<int32_t>(ops.size()));
}
