// Parser, printer and packer of term programs.
//
// Packing strategy (what the kernels rely on):
//
//  * Every node factor takes one of two values 1 + w^{v0} (form = 0) and 1 + w^{v1}
//    (form = 1).  The product of all factors therefore depends only on how many factors
//    currently sit in each value class k (value 1 + w^k).  With n_k those counts:
//        prod_k (1 + w^k)^{n_k} = w^R * sqrt2^E * Q(A - B)      if n_4 = 0, else 0,
//    because 1 + w^2 = sqrt2 w, 1 + w^6 = sqrt2 w^-1, 1 + w^7 = w^-1 (1 + w),
//    1 + w^5 = w^-3 (1 + w^3) and (1 + w)(1 + w^3) = sqrt2 w^2, where
//        A = n1 + n7,  B = n3 + n5,  m = min(A, B),
//        E = 2 n0 + n2 + n6 + m,     R = n2 - n6 - n7 - 3 n5 + 2 m   (mod 8),
//        Q(d) = (1 + w)^d for d >= 0 and (1 + w^3)^(-d) for d < 0.
//    Each of A, B, E, R is affine in the form bits, so it is a base value plus weighted
//    popcounts of L(x) against a few masks.  A small table holds w^r sqrt2^e Q(d) exactly.
//  * Linear phase terms c * l(x) are added to R the same way.
//  * A phase-pair factor (Eq. 3) is the sum over one extra Boolean z of
//        w^{z (b + 4 l2)} (1 + w^{a + 4 (l1 xor z)}),
//    and 4 z l2 = 2 z + 2 l2 - 2 (z xor l2) (mod 8), so it becomes a node factor and three
//    linear phase terms in one more parameter; those extra parameters are always walked
//    inside a slice, so slices still partition the original 2^p assignments.
//  * Factors on constant forms, and factors whose two values coincide, are multiplied
//    into the constant c at pack time (exactly, with overflow checks).
//  * Variable monomials are kept for a Gray-code walk: the parameters with the fewest
//    monomials are walked inside each slice, and each walk step adds only the change of
//    the monomials that contain the flipped parameter.

#include "program.h"

#include <array>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <sstream>

#include "../../include/zxpar.h"

// ------------------------------------------------------------------ IR text

namespace {

struct Lexer {
    std::vector<std::pair<std::string, int>> toks;  // token, line
    size_t pos = 0;
};

void lex(const char *text, size_t len, Lexer *lx) {
    int line = 1;
    size_t i = 0;
    while (i < len) {
        char ch = text[i];
        if (ch == '#') {
            while (i < len && text[i] != '\n') ++i;
        } else if (ch == '\n') {
            ++line;
            ++i;
        } else if (ch == ' ' || ch == '\t' || ch == '\r' || ch == '\f' || ch == '\v' || ch == '\0') {
            ++i;
        } else {
            size_t j = i;
            while (j < len && !strchr(" \t\r\n\f\v#", text[j]) && text[j] != '\0') ++j;
            lx->toks.emplace_back(std::string(text + i, j - i), line);
            i = j;
        }
    }
}

struct ParseError {
    std::string msg;
};

const std::pair<std::string, int> &next(Lexer *lx) {
    if (lx->pos >= lx->toks.size()) throw ParseError{"unexpected end of program text"};
    return lx->toks[lx->pos++];
}

void expect(Lexer *lx, const char *w) {
    const auto &t = next(lx);
    if (t.first != w)
        throw ParseError{"line " + std::to_string(t.second) + ": expected '" + w + "', got '" + t.first + "'"};
}

long long get_int(Lexer *lx, long long lo, long long hi) {
    const auto &t = next(lx);
    char *end = nullptr;
    errno = 0;
    long long v = strtoll(t.first.c_str(), &end, 10);
    if (*end || errno || t.first.empty())
        throw ParseError{"line " + std::to_string(t.second) + ": bad integer '" + t.first + "'"};
    if (v < lo || v > hi)
        throw ParseError{"line " + std::to_string(t.second) + ": value " + t.first + " out of range"};
    return v;
}

i128 get_i128(Lexer *lx) {
    const auto &t = next(lx);
    const char *s = t.first.c_str();
    bool neg = false;
    if (*s == '-') {
        neg = true;
        ++s;
    }
    if (!*s) throw ParseError{"line " + std::to_string(t.second) + ": bad integer"};
    i128 v = 0;
    for (; *s; ++s) {
        if (*s < '0' || *s > '9') throw ParseError{"line " + std::to_string(t.second) + ": bad integer"};
        if (__builtin_mul_overflow(v, (i128)10, &v) || __builtin_add_overflow(v, (i128)(*s - '0'), &v))
            throw ParseError{"line " + std::to_string(t.second) + ": constant exceeds int128"};
    }
    return neg ? -v : v;
}

uint64_t get_hex(Lexer *lx) {
    const auto &t = next(lx);
    char *end = nullptr;
    errno = 0;
    unsigned long long v = strtoull(t.first.c_str(), &end, 16);
    if (*end || errno || t.first.empty() || t.first[0] == '-')
        throw ParseError{"line " + std::to_string(t.second) + ": bad hex mask '" + t.first + "'"};
    return (uint64_t)v;
}

std::string i128_str(i128 v) {
    if (v == 0) return "0";
    bool neg = v < 0;
    unsigned __int128 u = neg ? (unsigned __int128)(-(v + 1)) + 1 : (unsigned __int128)v;
    std::string s;
    while (u) {
        s.push_back((char)('0' + (int)(u % 10)));
        u /= 10;
    }
    if (neg) s.push_back('-');
    std::reverse(s.begin(), s.end());
    return s;
}

}  // namespace

bool ir_parse(const char *text, size_t len, IrProgram *out, std::string *err) {
    Lexer lx;
    lex(text, len, &lx);
    IrProgram P;
    try {
        expect(&lx, "zxir");
        if (get_int(&lx, 1, 1) != 1) throw ParseError{"unsupported IR version"};
        expect(&lx, "p");
        P.p = (int)get_int(&lx, 0, 62);
        if (lx.pos < lx.toks.size() && lx.toks[lx.pos].first == "outer") {
            ++lx.pos;
            P.outer = (int)get_int(&lx, 0, P.p);
        }
        expect(&lx, "forms");
        long long nf = get_int(&lx, 0, 1 << 20);
        for (long long i = 0; i < nf; ++i) {
            expect(&lx, "f");
            IrForm f;
            f.cst = (int)get_int(&lx, 0, 1);
            f.mask = get_hex(&lx);
            if (P.p < 64 && (f.mask >> P.p)) throw ParseError{"form " + std::to_string(i) + " names a parameter >= p"};
            P.forms.push_back(f);
        }
        auto form_idx = [&](void) { return (int)get_int(&lx, 0, (long long)P.forms.size() - 1); };
        expect(&lx, "nodes");
        long long nn = get_int(&lx, 0, 1 << 20);
        for (long long i = 0; i < nn; ++i) {
            expect(&lx, "n");
            IrNode n;
            n.form = form_idx();
            n.a = (int)get_int(&lx, -(1LL << 30), 1LL << 30);
            n.b = (int)get_int(&lx, -(1LL << 30), 1LL << 30);
            P.nodes.push_back(n);
        }
        expect(&lx, "pairs");
        long long nq = get_int(&lx, 0, 1 << 20);
        for (long long i = 0; i < nq; ++i) {
            expect(&lx, "q");
            IrPair q;
            q.f1 = form_idx();
            q.f2 = form_idx();
            q.a = (int)get_int(&lx, -(1LL << 30), 1LL << 30);
            q.b = (int)get_int(&lx, -(1LL << 30), 1LL << 30);
            P.pairs.push_back(q);
        }
        expect(&lx, "lin");
        long long nl = get_int(&lx, 0, 1 << 20);
        for (long long i = 0; i < nl; ++i) {
            expect(&lx, "l");
            IrLin l;
            l.c = (int)get_int(&lx, -(1LL << 30), 1LL << 30);
            l.form = form_idx();
            P.lin.push_back(l);
        }
        expect(&lx, "mono");
        long long nm = get_int(&lx, 0, 1 << 20);
        for (long long i = 0; i < nm; ++i) {
            expect(&lx, "m");
            IrMono m;
            m.c = (int)get_int(&lx, -(1LL << 30), 1LL << 30);
            int d = (int)get_int(&lx, 1, 16);
            for (int k = 0; k < d; ++k) m.vars.push_back((int)get_int(&lx, 0, P.p - 1));
            P.mono.push_back(m);
        }
        expect(&lx, "scalar");
        for (int k = 0; k < 4; ++k) P.scalar.c[k] = get_i128(&lx);
        P.e = (int32_t)get_int(&lx, -(1LL << 30), 1LL << 30);
        expect(&lx, "end");
        if (lx.pos != lx.toks.size())
            throw ParseError{"line " + std::to_string(lx.toks[lx.pos].second) + ": text after 'end'"};
    } catch (const ParseError &pe) {
        if (err) *err = "IR: " + pe.msg;
        return false;
    }
    *out = std::move(P);
    return true;
}

std::string ir_print(const IrProgram &P) {
    std::ostringstream os;
    os << "zxir 1\np " << P.p << "\n";
    if (P.outer) os << "outer " << P.outer << "\n";
    os << "forms " << P.forms.size() << "\n";
    for (const auto &f : P.forms) os << "f " << f.cst << " " << std::hex << f.mask << std::dec << "\n";
    os << "nodes " << P.nodes.size() << "\n";
    for (const auto &n : P.nodes) os << "n " << n.form << " " << n.a << " " << n.b << "\n";
    os << "pairs " << P.pairs.size() << "\n";
    for (const auto &q : P.pairs) os << "q " << q.f1 << " " << q.f2 << " " << q.a << " " << q.b << "\n";
    os << "lin " << P.lin.size() << "\n";
    for (const auto &l : P.lin) os << "l " << l.c << " " << l.form << "\n";
    os << "mono " << P.mono.size() << "\n";
    for (const auto &m : P.mono) {
        os << "m " << m.c << " " << m.vars.size();
        for (int v : m.vars) os << " " << v;
        os << "\n";
    }
    os << "scalar";
    for (int k = 0; k < 4; ++k) os << " " << i128_str(P.scalar.c[k]);
    os << " " << P.e << "\nend\n";
    return os.str();
}

// ------------------------------------------------------------------ value table

Zw table_value(int d, int r, int e) {
    Zw z = zw_one();
    if (d >= 0) {
        for (int i = 0; i < d; ++i) z = zw_add(z, zw_rot(z, 1));  // times (1 + w)
    } else {
        for (int i = 0; i < -d; ++i) z = zw_add(z, zw_rot(z, 3));  // times (1 + w^3)
    }
    z = zw_rot(z, r);
    if (e) z = zw_times_sqrt2(z);
    return z;
}

// ------------------------------------------------------------------ packer

namespace {

// per value class k of a factor (value 1 + w^k): its contribution to A, B, E and R
int cls_A(int k) { return (k == 1 || k == 7) ? 1 : 0; }
int cls_B(int k) { return (k == 3 || k == 5) ? 1 : 0; }
int cls_E(int k) { return k == 0 ? 2 : ((k == 2 || k == 6) ? 1 : 0); }
int cls_R(int k) {
    switch (k) {
        case 2: return 1;
        case 6: return -1;
        case 7: return -1;
        case 5: return -3;
        default: return 0;
    }
}

int mod8(long long v) { return (int)(((v % 8) + 8) % 8); }

struct Work {
    int pe = 0;
    std::vector<IrForm> forms;  // masks over eval variables (pair variables first)
    std::vector<std::pair<int, std::pair<int, int>>> nodes;  // form, (v0, v1)
    std::vector<std::pair<int, int>> lin;                    // (c mod 8, form)
    std::map<std::vector<int>, int> mono;                    // sorted vars -> c mod 8
    Zw c0;
    int32_t e = 0;
    bool zero = false;
};

bool mul_const(Work *w, const Zw &f, std::string *err) {
    Zw r;
    if (!zw_mul_checked(w->c0, f, &r)) {
        *err = "constant factor exceeds int128";
        return false;
    }
    w->c0 = r;
    zw_canonicalise(&w->c0, &w->e);
    if (zw_is_zero(w->c0)) w->zero = true;
    return true;
}

Zw one_plus_w(int k) {
    Zw z = zw_rot(zw_one(), k);
    z.c[0] += 1;
    return z;
}

}  // namespace

// Fraction of assignments on which no node factor vanishes.  A factor with values (v0, v1) on
// its form l vanishes where l takes the value whose exponent is 4 (1 + w^4 = 0), so the
// surviving assignments satisfy one affine equation per such factor: an affine subspace of
// codimension rank (Gaussian elimination over GF(2)), or none if the equations contradict.
static double nonzero_fraction(const std::vector<IrForm> &forms, const std::vector<std::pair<int, std::pair<int, int>>> &nodes) {
    std::vector<std::pair<uint64_t, int>> rows;  // mask . x = rhs
    for (const auto &n : nodes) {
        const IrForm &f = forms[n.first];
        const int v0 = n.second.first, v1 = n.second.second;
        if (v0 != 4 && v1 != 4) continue;
        const int need = v0 == 4 ? 1 : 0;  // the value of l that keeps the factor non-zero
        rows.push_back({f.mask, need ^ (int)f.cst});
    }
    int rank = 0;
    for (size_t r = 0; r < rows.size(); ++r) {
        uint64_t m = rows[r].first;
        int rhs = rows[r].second;
        if (!m) {
            if (rhs) return 0.0;
            continue;
        }
        const uint64_t piv = m & (~m + 1);
        for (size_t t = r + 1; t < rows.size(); ++t)
            if (rows[t].first & piv) {
                rows[t].first ^= m;
                rows[t].second ^= rhs;
            }
        ++rank;
    }
    return std::ldexp(1.0, -rank);
}

// ---- exact elimination of the vanishing conditions
//
// A node factor 1 + w^{a + b l(x)} with a = 4 or a + b = 4 (mod 8) is zero at one value of its
// form (1 + w^4 = 0: the factor kills the term, Section 5), so every term that survives has
// l(x) = keep, one affine equation over GF(2) per such factor.  Gaussian elimination solves them
// for `rank` pivot parameters (never a query parameter; among a condition's parameters the one
// met by the fewest monomials of degree >= 2), and substituting x_v = r_v XOR <m_v, x> (m_v over
// the free parameters) restricts the sum to the surviving affine subspace: the 2^(p - rank)
// assignments of the free parameters.  Forms stay affine forms (the vanishing factors' forms
// become the constant `keep`, so they fold into the program constant); a variable monomial with
// a pivot becomes a product of affine forms (a form monomial), or a linear term or a variable
// monomial again when its forms reduce to one form or to plain parameters.  The sum is the same
// number: the eliminated terms are exactly the zero ones.
//
// Returns false (nothing changed) when the program has no vanishing factor, has pair factors, a
// condition involves query parameters only, or the form monomials would use more than
// kMaxMonoForms distinct forms.
struct Elimination {
    int rank = 0;
    std::vector<int> free_orig;  // new parameter j is original parameter free_orig[j]
    uint64_t x0 = 0;             // the assignment of the given parameters at t = 0
    std::vector<uint64_t> cols;  // ... and what new parameter j = 1 adds to it
};
constexpr int kMaxMonoForms = 32;
// programs of at most 2^kFormMonoMaxParams terms evaluate their variable monomials as form
// monomials (about 1024 blocks of 64 lanes x 64 terms: one wave per SIMD)
constexpr int kFormMonoMaxParams = 22;

static bool eliminate_vanishing(const IrProgram &ir, IrProgram *red, std::vector<IrFormMono> *fmono,
                                Elimination *el) {
    if (!ir.pairs.empty() || ir.p == 0) return false;
    const int p = ir.p;
    std::vector<std::pair<uint64_t, int>> rows;  // parity(mask & x) = rhs
    for (const auto &n : ir.nodes) {
        const IrForm &f = ir.forms[n.form];
        const int v0 = mod8(n.a), v1 = mod8((long long)n.a + n.b);
        if (f.mask == 0 || v0 == v1 || (v0 != 4 && v1 != 4)) continue;
        const int keep = v0 == 4 ? 1 : 0;
        rows.push_back({f.mask, keep ^ f.cst});
    }
    if (rows.empty()) return false;
    std::vector<int> inc(p, 0);
    for (const auto &m : ir.mono)
        if (m.vars.size() >= 2)
            for (int v : m.vars) inc[v]++;
    const int inner_p = p - ir.outer;
    const uint64_t eligible = inner_p >= 64 ? ~0ull : (((uint64_t)1 << inner_p) - 1);
    std::vector<std::pair<uint64_t, int>> R;  // reduced rows: each pivot bit in its own row only
    std::vector<int> pv;
    bool contradiction = false;
    for (auto r : rows) {
        uint64_t m = r.first;
        int rhs = r.second;
        for (size_t i = 0; i < R.size(); ++i)
            if (m >> pv[i] & 1) {
                m ^= R[i].first;
                rhs ^= R[i].second;
            }
        if (!m) {
            if (rhs) contradiction = true;
            continue;
        }
        const uint64_t cand = m & eligible;
        if (!cand) return false;
        int best = -1;
        for (uint64_t c = cand; c; c &= c - 1) {
            const int v = __builtin_ctzll(c);
            if (best < 0 || inc[v] < inc[best]) best = v;
        }
        for (size_t i = 0; i < R.size(); ++i)
            if (R[i].first >> best & 1) {
                R[i].first ^= m;
                R[i].second ^= rhs;
            }
        R.push_back({m, rhs});
        pv.push_back(best);
    }
    *red = IrProgram();
    *fmono = {};
    *el = Elimination();
    if (contradiction) {  // no assignment survives: the sum is zero
        *red = ir;
        red->scalar = zw_zero();
        red->e = 0;
        el->free_orig.resize(p);
        for (int i = 0; i < p; ++i) {
            el->free_orig[i] = i;
            el->cols.push_back((uint64_t)1 << i);
        }
        return true;
    }
    uint64_t pivots = 0;
    std::vector<IrForm> sub(p);  // each parameter as an affine form of the free parameters
    for (int i = 0; i < p; ++i) sub[i] = IrForm{0, (uint64_t)1 << i};
    for (size_t i = 0; i < R.size(); ++i) {
        pivots |= (uint64_t)1 << pv[i];
        sub[pv[i]] = IrForm{R[i].second, R[i].first & ~((uint64_t)1 << pv[i])};
    }
    std::vector<int> new_of(p, -1);
    for (int i = 0; i < p; ++i)
        if (!(pivots >> i & 1)) {
            new_of[i] = (int)el->free_orig.size();
            el->free_orig.push_back(i);
        }
    el->rank = (int)R.size();
    for (int u : el->free_orig) {
        uint64_t col = (uint64_t)1 << u;
        for (size_t i = 0; i < R.size(); ++i)
            if (sub[pv[i]].mask >> u & 1) col |= (uint64_t)1 << pv[i];
        el->cols.push_back(col);
    }
    for (size_t i = 0; i < R.size(); ++i)
        if (sub[pv[i]].cst) el->x0 |= (uint64_t)1 << pv[i];
    auto substitute = [&](const IrForm &f) {  // over original free parameters
        IrForm g{f.cst, f.mask & ~pivots};
        for (uint64_t b = f.mask & pivots; b; b &= b - 1) {
            const IrForm &s = sub[__builtin_ctzll(b)];
            g.cst ^= s.cst;
            g.mask ^= s.mask;
        }
        return g;
    };
    auto remap = [&](uint64_t m) {
        uint64_t r = 0;
        for (; m; m &= m - 1) r |= (uint64_t)1 << new_of[__builtin_ctzll(m)];
        return r;
    };
    red->p = p - el->rank;
    red->outer = ir.outer;
    for (const auto &f : ir.forms) {
        const IrForm g = substitute(f);
        red->forms.push_back(IrForm{g.cst, remap(g.mask)});
    }
    red->nodes = ir.nodes;
    red->lin = ir.lin;
    red->scalar = ir.scalar;
    red->e = ir.e;
    std::vector<IrForm> mforms;  // distinct forms of the form monomials
    for (const auto &m : ir.mono) {
        bool has_pivot = false;
        for (int v : m.vars) has_pivot = has_pivot || (pivots >> v & 1);
        if (!has_pivot) {
            IrMono nm{m.c, {}};
            for (int v : m.vars) nm.vars.push_back(new_of[v]);
            red->mono.push_back(nm);
            continue;
        }
        // the product of the substituted forms, as 0/1 values: drop factors 1, stop at a factor 0,
        // l * l = l, l * (1 xor l) = 0
        std::vector<IrForm> fs;
        bool zero = false;
        for (int v : m.vars) {
            const IrForm g = sub[v];
            if (g.mask == 0) {
                if (!g.cst) zero = true;
                continue;
            }
            bool dup = false;
            for (const auto &h : fs)
                if (h.mask == g.mask) {
                    dup = true;
                    if (h.cst != g.cst) zero = true;
                }
            if (!dup) fs.push_back(g);
        }
        if (zero) continue;
        if (fs.empty()) {  // the constant c: a linear term on a constant form
            red->forms.push_back(IrForm{1, 0});
            red->lin.push_back(IrLin{m.c, (int)red->forms.size() - 1});
            continue;
        }
        if (fs.size() == 1) {
            red->forms.push_back(IrForm{fs[0].cst, remap(fs[0].mask)});
            red->lin.push_back(IrLin{m.c, (int)red->forms.size() - 1});
            continue;
        }
        bool plain = true;
        for (const auto &h : fs) plain = plain && h.cst == 0 && __builtin_popcountll(h.mask) == 1;
        if (plain) {
            IrMono nm{m.c, {}};
            for (const auto &h : fs) nm.vars.push_back(new_of[__builtin_ctzll(h.mask)]);
            red->mono.push_back(nm);
            continue;
        }
        IrFormMono fm{m.c, {}};
        for (const auto &h : fs) {
            const IrForm r{h.cst, remap(h.mask)};
            fm.forms.push_back(r);
            bool seen = false;
            for (const auto &q : mforms) seen = seen || (q.cst == r.cst && q.mask == r.mask);
            if (!seen) mforms.push_back(r);
        }
        fmono->push_back(fm);
    }
    if ((int)mforms.size() > kMaxMonoForms) return false;
    return true;
}

// Which parameters are walked, and in what order (walk position q + j for walked[j]), decides
// the walk's per-block work on variable monomials: a monomial costs work at each flip of one
// of its outer walk positions i >= KB, an entry of the flip list when it also needs walk bits
// above i, an inner-vector entry (about three times the work) when it also has an inner
// variable, and position i flips once every 2^(i - KB + 1) blocks.  Starting from the given
// order, swaps of two walked parameters, or of a walked and an unwalked one (never a query
// parameter), are kept while that estimate drops.  The order changes no term's value.
std::vector<int> refine_walk_order(const Work &w, int p, int q, int inner_p, std::vector<int> walked) {
    const int g_orig = (int)walked.size();
    if (w.mono.empty() || g_orig < 2) return walked;
    // the form-vector width, hence the inner bits, does not depend on the order: every node
    // factor owns a bit and linear terms share the bits of their forms
    std::vector<char> node_form(w.forms.size(), 0), lin_bit(w.forms.size(), 0);
    int F = (int)w.nodes.size();
    for (const auto &n : w.nodes) node_form[n.first] = 1;
    for (const auto &l : w.lin)
        if (!node_form[l.second] && !lin_bit[l.second]) {
            lin_bit[l.second] = 1;
            ++F;
        }
    int Wd = 1;
    while (Wd * 32 < F) Wd *= 2;
    const int KB = inner_bits_for((uint32_t)Wd);
    if (q + g_orig <= KB) return walked;
    std::vector<std::vector<int>> mv;
    for (const auto &m : w.mono) {
        std::vector<int> vs;
        for (int v : m.first) vs.push_back(v - q);
        mv.push_back(vs);
    }
    std::vector<int> wpos(p, -1);
    auto cost = [&](const std::vector<int> &wk) {
        for (size_t j = 0; j < wk.size(); ++j) wpos[wk[j]] = q + (int)j;
        const int G = q + (int)wk.size();
        const uint32_t inner_mask = (1u << KB) - 1;
        double c = 0;
        for (const auto &vs : mv) {
            uint32_t M = 0;
            for (int v : vs)
                if (wpos[v] >= 0) M |= 1u << wpos[v];
            const uint32_t inner = M & inner_mask;
            for (int i = KB; i < G; ++i) {
                if (!(M >> i & 1)) continue;
                const double freq = std::ldexp(1.0, -(i - KB + 1));
                const uint32_t others = M & ~(1u << i);
                const uint32_t below = (1u << (i - 1)) - 1;
                if (!(others & below) && (others >> (i + 1))) c += freq;  // flip-list entry
                if (inner) {
                    const uint32_t other = others & ~inner_mask;
                    const uint32_t clear_below = i - 1 > KB ? ((1u << (i - 1)) - 1) & ~inner_mask : 0u;
                    if (!(other & clear_below)) c += 3.0 * freq;  // inner-vector entry
                }
            }
        }
        for (int v : wk) wpos[v] = -1;
        return c;
    };
    std::vector<char> in_walk(p, 0);
    for (int v : walked) in_walk[v] = 1;
    std::vector<int> pool;
    for (int v = 0; v < inner_p; ++v)
        if (!in_walk[v]) pool.push_back(v);
    double best = cost(walked);
    for (int pass = 0; pass < 32; ++pass) {
        bool improved = false;
        for (int a = 0; a < g_orig; ++a) {
            for (int b = a + 1; b < g_orig; ++b) {
                std::swap(walked[a], walked[b]);
                const double c = cost(walked);
                if (c < best - 1e-12) {
                    best = c;
                    improved = true;
                } else {
                    std::swap(walked[a], walked[b]);
                }
            }
            for (size_t u = 0; u < pool.size(); ++u) {
                std::swap(walked[a], pool[u]);
                const double c = cost(walked);
                if (c < best - 1e-12) {
                    best = c;
                    improved = true;
                } else {
                    std::swap(walked[a], pool[u]);
                }
            }
        }
        if (!improved) break;
    }
    return walked;
}

int pack_program(const IrProgram &ir_given, int max_walk_bits, PackedProgram *out, std::string *err,
                 bool eliminate) {
    PackedProgram &P = *out;
    P = PackedProgram();
    IrProgram reduced;
    std::vector<IrFormMono> fmono;
    Elimination elim;
    const bool eliminated = eliminate && eliminate_vanishing(ir_given, &reduced, &fmono, &elim);
    const IrProgram &ir = eliminated ? reduced : ir_given;
    P.p_given = ir_given.p;
    P.eliminated = eliminated ? elim.rank : 0;
    P.p = ir.p;
    P.q = (int)ir.pairs.size();
    Work w;
    w.pe = ir.p + P.q;
    if (w.pe > 62) {
        *err = "too many parameters (p plus pair factors must be <= 62)";
        return SIM_ERANGE;
    }
    w.c0 = ir.scalar;
    w.e = ir.e;
    zw_canonicalise(&w.c0, &w.e);
    if (zw_is_zero(w.c0)) w.zero = true;
    const int q = P.q;

    // forms over eval variables: pair variable k is bit k, original parameter i is bit q + i
    for (const auto &f : ir.forms) w.forms.push_back(IrForm{f.cst, f.mask << q});
    int const_phase = 0;
    for (const auto &n : ir.nodes) {
        const IrForm &f = w.forms[n.form];
        int v0 = mod8(n.a), v1 = mod8((long long)n.a + n.b);
        if (f.mask == 0 || v0 == v1) {
            if (!mul_const(&w, one_plus_w(f.cst ? v1 : v0), err)) return SIM_ERANGE;
        } else {
            w.nodes.push_back({n.form, {v0, v1}});
        }
    }
    // Two node factors on the same parity (equal masks; a constant of 1 swaps a factor's two
    // values) whose product is the same at both values of the parity are that constant: the
    // pairwise cancellation of node subterms whose constants differ by pi that the paper leaves
    // for future work (Section 5), applied to every program.  1 + w^0 with 1 + w^4 on one parity
    // makes the whole program zero.
    {
        std::vector<char> gone(w.nodes.size(), 0);
        auto oriented = [&](size_t i) {  // the factor's exponents at <mask, x> = 0 and = 1
            const auto &n = w.nodes[i];
            return w.forms[n.first].cst ? std::make_pair(n.second.second, n.second.first) : n.second;
        };
        for (size_t i = 0; i < w.nodes.size(); ++i) {
            if (gone[i]) continue;
            const uint64_t mi = w.forms[w.nodes[i].first].mask;
            const auto vi = oriented(i);
            for (size_t j = i + 1; j < w.nodes.size(); ++j) {
                if (gone[j] || w.forms[w.nodes[j].first].mask != mi) continue;
                const auto vj = oriented(j);
                Zw at0, at1;
                if (!zw_mul_checked(one_plus_w(vi.first), one_plus_w(vj.first), &at0) ||
                    !zw_mul_checked(one_plus_w(vi.second), one_plus_w(vj.second), &at1))
                    continue;
                bool same = true;
                for (int k = 0; k < 4; ++k) same = same && at0.c[k] == at1.c[k];
                if (!same) continue;
                if (!mul_const(&w, at0, err)) return SIM_ERANGE;
                gone[i] = gone[j] = 1;
                break;
            }
        }
        std::vector<std::pair<int, std::pair<int, int>>> kept;
        for (size_t i = 0; i < w.nodes.size(); ++i)
            if (!gone[i]) kept.push_back(w.nodes[i]);
        w.nodes.swap(kept);
    }
    for (int k = 0; k < q; ++k) {
        const IrPair &pr = ir.pairs[k];
        uint64_t zbit = (uint64_t)1 << k;
        const IrForm f1 = w.forms[pr.f1], f2 = w.forms[pr.f2];
        int fz1 = (int)w.forms.size();
        w.forms.push_back(IrForm{f1.cst, f1.mask ^ zbit});
        int fz = (int)w.forms.size();
        w.forms.push_back(IrForm{0, zbit});
        int fz2 = (int)w.forms.size();
        w.forms.push_back(IrForm{f2.cst, f2.mask ^ zbit});
        int v0 = mod8(pr.a), v1 = mod8((long long)pr.a + 4);
        w.nodes.push_back({fz1, {v0, v1}});
        w.lin.push_back({mod8((long long)pr.b + 2), fz});  // (b + 2) z
        if (f2.mask == 0) const_phase += 2 * f2.cst;        // 2 l2
        else w.lin.push_back({2, pr.f2});
        w.lin.push_back({6, fz2});                          // -2 (z xor l2)
    }
    for (const auto &m : ir.mono) {
        std::vector<int> vs;
        for (int v : m.vars) vs.push_back(v + q);
        std::sort(vs.begin(), vs.end());
        vs.erase(std::unique(vs.begin(), vs.end()), vs.end());
        int &c = w.mono[vs];
        c = mod8((long long)c + m.c);
    }
    for (auto it = w.mono.begin(); it != w.mono.end();) {
        if (it->second == 0) it = w.mono.erase(it);
        else ++it;
    }
    // Small programs (a few thousand blocks of terms: about one wave per SIMD): the per-slice
    // set-up of the variable monomials' walk lists would cost more than the blocks themselves, so
    // every variable monomial becomes a form monomial over coordinate forms (evaluated per block,
    // nothing per slice), and those of degree one linear terms on their coordinate forms.
    std::vector<IrLin> extra_lin;
    bool fm_only = false;  // the variable monomials became form monomials
    {
        // (only without factors that can vanish: the walks that test them per block do not
        // evaluate form monomials)
        bool conv = q == 0 && !w.mono.empty() && w.pe <= kFormMonoMaxParams;
        for (const auto &n : w.nodes) conv = conv && n.second.first != 4 && n.second.second != 4;
        std::vector<IrForm> seen;
        auto note = [&](const IrForm &f) {
            for (const auto &h : seen)
                if (h.cst == f.cst && h.mask == f.mask) return;
            seen.push_back(f);
        };
        for (const auto &m : fmono)
            for (const auto &f : m.forms) note(f);
        for (const auto &m : w.mono) {
            if (m.first.size() > 3) conv = false;
            if (m.first.size() >= 2)
                for (int v : m.first) note(IrForm{0, (uint64_t)1 << v});
        }
        for (const auto &m : w.mono)
            if (m.first.size() == 1) note(IrForm{0, (uint64_t)1 << m.first[0]});
        if (conv && (int)seen.size() <= kMaxMonoForms) {
            fm_only = true;
            // (a degree-one monomial is a form monomial whose one form is taken twice)
            for (const auto &m : w.mono) {
                IrFormMono fm{m.second, {}};
                for (int v : m.first) fm.forms.push_back(IrForm{0, (uint64_t)1 << v});
                if (fm.forms.size() == 1) fm.forms.push_back(fm.forms[0]);
                fmono.push_back(fm);
            }
            w.mono.clear();
        }
    }
    std::vector<IrLin> all_lin = ir.lin;
    all_lin.insert(all_lin.end(), extra_lin.begin(), extra_lin.end());
    for (const auto &l : all_lin) {
        int c = mod8(l.c);
        if (!c) continue;
        const IrForm &f = w.forms[l.form];
        if (f.mask == 0) const_phase += c * f.cst;
        else w.lin.push_back({c, l.form});
    }
    // The weight-4 parts of the linear phase terms are one term: w^(4 (f_1 + ... + f_m)) =
    // (-1)^(f_1 xor ... xor f_m), and the xor of affine forms over GF(2) is one affine form.
    // Every other form keeps its coefficient mod 4.  The combined term comes first, so its bit
    // of L is the first after the node bits, where the node table can carry it.
    {
        std::vector<int> seen;
        std::map<int, long long> tot;
        for (const auto &l : w.lin) {
            if (!tot.count(l.second)) seen.push_back(l.second);
            tot[l.second] += l.first;
        }
        IrForm g{0, 0};
        bool any4 = false;
        std::vector<std::pair<int, int>> lin;
        for (int f : seen) {
            const int t = mod8(tot[f]);
            if (t & 4) {
                g.cst ^= w.forms[f].cst;
                g.mask ^= w.forms[f].mask;
                any4 = true;
            }
            if (t & 3) lin.push_back({t & 3, f});
        }
        if (any4 && g.mask == 0) {
            const_phase += 4 * g.cst;
        } else if (any4) {
            int fg = -1;
            for (size_t f = 0; f < w.forms.size() && fg < 0; ++f)
                if (w.forms[f].mask == g.mask) {
                    fg = (int)f;
                    if (w.forms[f].cst != g.cst) const_phase += 4;  // (-1)^(f xor 1) = -(-1)^f
                }
            if (fg < 0) {
                fg = (int)w.forms.size();
                w.forms.push_back(g);
            }
            lin.insert(lin.begin(), {4, fg});
        }
        w.lin.swap(lin);
    }
    if (mod8(const_phase)) w.c0 = zw_rot(w.c0, mod8(const_phase));
    if (w.zero) {
        w.c0 = zw_zero();
        w.e = 0;
    }

    // ---- packed order of the eval variables
    const int p = ir.p;
    std::vector<int> inc(p, 0);  // monomial incidences per original parameter
    for (const auto &m : w.mono)
        for (int v : m.first) inc[v - q]++;
    // Walk length: a slice costs a set-up (its high parameters into L, and with variable
    // monomials a full evaluation of phi) that the 2^g walk steps amortise; without variable
    // monomials the set-up is a few XORs per high parameter.  The kernels balance work in
    // blocks of a walk, so long walks cost no balance, but a wave holds 64 slices, so the walk
    // leaves at least 64 slices where the program is large enough.
    const bool any_mono = !w.mono.empty() || !fmono.empty();
    const int want = any_mono ? 12 : 8;
    const int inner_p = p - ir.outer;  // query parameters are never walked
    int g_orig = std::min(inner_p, std::min(max_walk_bits, want));
    if (p - g_orig < 6) g_orig = std::max(std::min(inner_p, kMaxInnerBits), p - 6);
    g_orig = std::min(g_orig, inner_p);
    if (any_mono) g_orig = std::min(g_orig, std::max(0, 16 - q));  // packed 4-bit fields
    if (p - g_orig > 62) g_orig = p - 62;
    if (any_mono && q + g_orig > 16) {
        *err = "too many pair factors together with variable monomials (at most 16 walk bits)";
        return SIM_ERANGE;
    }
    // walked parameters: fewest monomials first (they flip most often); high: index order, so
    // the query parameters (the last `outer`) are the top slice bits
    std::vector<int> order(inner_p);
    for (int i = 0; i < inner_p; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return inc[a] < inc[b]; });
    std::vector<int> walked(order.begin(), order.begin() + g_orig);
    std::sort(walked.begin(), walked.end(), [&](int a, int b) {
        return inc[a] != inc[b] ? inc[a] < inc[b] : a < b;
    });
    walked = refine_walk_order(w, p, q, inner_p, walked);
    std::vector<char> is_walked(p, 0);
    for (int v : walked) is_walked[v] = 1;
    std::vector<int> pos_of(w.pe, -1);  // eval variable -> packed position
    for (int k = 0; k < q; ++k) pos_of[k] = k;
    int pos = q;
    P.perm.clear();
    for (int v : walked) {
        pos_of[v + q] = pos++;
        P.perm.push_back(v);
    }
    for (int i = 0; i < p; ++i)
        if (!is_walked[i]) {
            pos_of[i + q] = pos++;
            P.perm.push_back(i);
        }
    const int g = q + g_orig;
    if (g > 24) {
        *err = "too many pair factors for one Gray walk (walk length at most 2^24)";
        return SIM_ERANGE;
    }
    P.walk_bits = g_orig;
    P.outer = ir.outer;
    P.n_slices = (uint64_t)1 << (w.pe - g);
    auto permute = [&](uint64_t m) {
        uint64_t r = 0;
        for (int v = 0; v < w.pe; ++v)
            if (m >> v & 1) r |= (uint64_t)1 << pos_of[v];
        return r;
    };
    // slice-ordered index -> assignment of the given parameters
    P.lay_cols.clear();
    P.lay_x0 = eliminated ? elim.x0 : 0;
    for (int j = 0; j < p; ++j) {
        const int v = P.perm[j];
        P.lay_cols.push_back(eliminated ? elim.cols[v] : (uint64_t)1 << v);
        if (eliminated) P.perm[j] = elim.free_orig[v];
    }
    // Form monomials: their distinct forms are bits 0 .. n_mf - 1 of a per-lane vector O.  At the
    // first term of a block, O = S ^ G ^ (odd block ? gcol[KB - 1] : 0): S per lane and slice (the
    // constants and slice parts), G the outer walk parts of the current walk state (updated with
    // gcol[i] at each flip of walk position i, wave-uniform).  At step k of the block a form is
    // its bit of O xor lambda bit k, lambda = its inner part's parity at gray(k).
    // entries grouped by degree (two forms, then three) and coefficient 1..7, so that the kernel
    // runs one branch-free loop per group; a zero coefficient contributes nothing
    {
        std::vector<IrFormMono> sorted;
        for (int d3 = 0; d3 < 2; ++d3)
            for (int c = 1; c < 8; ++c)
                for (const auto &m : fmono)
                    if ((m.forms.size() == 3) == (d3 == 1) && mod8(m.c) == c) sorted.push_back(m);
        fmono.swap(sorted);
    }
    std::vector<IrForm> mforms;
    std::vector<std::array<int, 3>> fm_idx;
    for (const auto &m : fmono) {
        std::array<int, 3> ix = {-1, -1, -1};
        for (size_t t = 0; t < m.forms.size(); ++t) {
            const IrForm f{m.forms[t].cst, permute(m.forms[t].mask)};
            int j = -1;
            for (size_t u = 0; u < mforms.size(); ++u)
                if (mforms[u].cst == f.cst && mforms[u].mask == f.mask) j = (int)u;
            if (j < 0) {
                j = (int)mforms.size();
                mforms.push_back(f);
            }
            ix[t] = j;
        }
        fm_idx.push_back(ix);
    }
    std::vector<uint32_t> gcol(g, 0);
    for (size_t j = 0; j < mforms.size(); ++j)
        for (int i = 0; i < g; ++i)
            if (mforms[j].mask >> i & 1) gcol[i] |= 1u << j;
    P.n_fmono = (int)fmono.size();
    P.n_mforms = (int)mforms.size();

    // ---- forms actually used, in packed positions
    // every node factor owns its bit of L (so its statistic weights are single steps);
    // linear phase terms share bits freely
    std::vector<int> form_slot(w.forms.size(), -1);
    std::vector<IrForm> used;
    std::vector<char> node_owned;
    auto new_bit = [&](int f) {
        used.push_back(IrForm{w.forms[f].cst, permute(w.forms[f].mask)});
        node_owned.push_back(0);
        return (int)used.size() - 1;
    };
    // factors that can vanish (1 + w^4 = 0 at one value of their form) first: their bits of L
    // are then the lowest ones, which lets a block look its surviving steps up by those bits
    std::stable_partition(w.nodes.begin(), w.nodes.end(), [](const std::pair<int, std::pair<int, int>> &n) {
        return n.second.first == 4 || n.second.second == 4;
    });
    for (auto &n : w.nodes) {
        int f = n.first;
        int b = form_slot[f];
        if (b < 0 || node_owned[b]) {
            b = new_bit(f);
            if (form_slot[f] < 0) form_slot[f] = b;
        }
        node_owned[b] = 1;
        n.first = b;
    }
    int lin4_bit = -1;  // the bit of the combined weight-4 phase term
    for (auto &l : w.lin) {
        int f = l.second;
        if (form_slot[f] < 0) form_slot[f] = new_bit(f);
        l.second = form_slot[f];
        if (l.first & 4) lin4_bit = l.second;
    }
    const int F = (int)used.size();
    int W = 1;
    while (W * 32 < F) W *= 2;
    if (W > 16) {
        *err = "too many distinct forms (at most 512)";
        return SIM_ERANGE;
    }
    P.W = W;
    const int KB = inner_bits_for((uint32_t)W);  // inner bits of a block
    const int KS = 1 << KB;                      // terms of a block
    const int NF = KS / 8;                       // words of a block's 4-bit phase fields
    P.n_forms = F;
    P.n_factors = (int)w.nodes.size();
    P.n_mono = (int)w.mono.size();

    // ---- static bound: every node factor has |sigma(F)| <= 2 in every embedding, so each
    // coefficient of a term is <= 2^nodes and the sum over 2^pe terms is <= 2^(nodes + pe)
    if (!w.zero && (long long)w.nodes.size() + w.pe > 125) {
        *err = "static bound exceeds int128 (factors + parameters > 125)";
        return SIM_ERANGE;
    }

    // ---- statistics
    std::vector<long long> wt[N_STATS];
    for (int s = 0; s < N_STATS; ++s) wt[s].assign(F, 0);
    long long base[N_STATS] = {0, 0, 0, 0};
    std::vector<uint32_t> zmask(W, 0), zflip(W, 0);
    bool has_zero = false;
    typedef int (*ClsFn)(int);
    ClsFn fns[N_STATS] = {cls_A, cls_B, cls_E, cls_R};
    long long amax = 0, amin = 0, bmax = 0, bmin = 0;
    for (const auto &n : w.nodes) {
        int f = n.first, v0 = n.second.first, v1 = n.second.second;
        for (int s = 0; s < N_STATS; ++s) {
            base[s] += fns[s](v0);
            wt[s][f] += fns[s](v1) - fns[s](v0);
        }
    }
    for (const auto &l : w.lin) wt[STAT_R][l.second] += l.first;
    std::vector<long long> wt_lin(F, 0);  // phase weights of the linear terms alone
    long long base_lin = 0;
    for (const auto &l : w.lin) wt_lin[l.second] += l.first;
    // Factors that can vanish (one value of their form gives 1 + w^4 = 0): on every term that
    // survives, their form takes the other value, so the statistic weights of their bit (the
    // factor's own, and those of linear terms sharing the bit) are constants folded into the
    // base.  Their bit of L is kept as "the factor vanishes" (the constant vector is
    // complemented where that happens at l = 0), so a term is zero iff L & zmask != 0.
    for (const auto &n : w.nodes) {
        const int f = n.first, v0 = n.second.first, v1 = n.second.second;
        if (v0 != 4 && v1 != 4) continue;
        const int keep = v0 == 4 ? 1 : 0;  // value of the form on surviving terms
        zmask[f / 32] |= 1u << (f % 32);
        if (v0 == 4) zflip[f / 32] |= 1u << (f % 32);
        has_zero = true;
        for (int s = 0; s < N_STATS; ++s) {
            base[s] += wt[s][f] * keep;
            wt[s][f] = 0;
        }
        base_lin += wt_lin[f] * keep;
        wt_lin[f] = 0;
    }
    for (int f = 0; f < F; ++f) {
        if (wt[STAT_A][f] > 0) amax += wt[STAT_A][f]; else amin += wt[STAT_A][f];
        if (wt[STAT_B][f] > 0) bmax += wt[STAT_B][f]; else bmin += wt[STAT_B][f];
    }
    amax += base[STAT_A];
    amin += base[STAT_A];
    bmax += base[STAT_B];
    bmin += base[STAT_B];
    amin = std::max(0LL, amin);
    bmin = std::max(0LL, bmin);
    long long dmin = amin - bmax, dmax = amax - bmin;
    if (dmax > 63 || dmin < -63) {
        *err = "more than 63 odd-class factors (table range)";
        return SIM_ERANGE;
    }
    if (dmin > dmax) dmin = dmax = 0;
    const int nd = (int)(dmax - dmin + 1);
    // accumulation mode: int64 registers when the static bound allows, else per-block class
    // counters when they fit the LDS budget, else int128 registers
    uint32_t acc_mode, q_limbs;
    bool flush128 = false;
    {
        long long emax = base[STAT_E];
        for (int f = 0; f < F; ++f)
            if (wt[STAT_E][f] > 0) emax += wt[STAT_E][f];
        emax += std::max(0LL, std::min(amax, bmax));
        const int hmax = (int)std::max(0LL, emax) / 2;
        q_limbs = (uint32_t)(hmax / 32 + 1);
        const long long bound_bits = (long long)w.nodes.size() + w.pe;
        const size_t class_bytes = (size_t)nd * 16 * q_limbs * 8;
        if (bound_bits <= 62) acc_mode = ACC_I64;
        // a block's 2^KB terms sum below 2^(nodes + KB) per coordinate: int64 within a block,
        // moved to int128 after it (walks of whole blocks without vanishing factors)
        else if (!has_zero && g >= KB && (long long)w.nodes.size() + KB <= 62) {
            acc_mode = ACC_I64;
            flush128 = true;
        } else if (class_bytes <= 48 * 1024) acc_mode = ACC_CLASS;
        else acc_mode = ACC_I128;
    }
    // node table: few node factors (their bits are 0 .. n-1, allocated first), W up to 8
    const int n_nodes = (int)w.nodes.size();
    bool use_ntab = n_nodes >= 1 && n_nodes <= kMaxTableNodes && acc_mode != ACC_I128 && W <= 8;
    for (int j = 0; j < n_nodes && use_ntab; ++j) use_ntab = w.nodes[j].first == j;
    // the table is indexed by the node bits and, when it follows them, the bit of the combined
    // weight-4 phase term; it carries every linear phase weight on those bits
    const int ntab_bits = n_nodes + (lin4_bit == n_nodes ? 1 : 0);
    std::vector<long long> wt_tab(use_ntab ? ntab_bits : 0, 0);

    // ---- image words
    std::vector<uint32_t> img;
    ImgHeader &H = P.hdr;
    memset(&H, 0, sizeof H);
    H.pe = (uint32_t)w.pe;
    H.g = (uint32_t)g;
    H.W = (uint32_t)W;
    H.has_zero = has_zero ? 1u : 0u;
    H.has_mono = any_mono ? 1u : 0u;
    H.n_slices_lo = (uint32_t)P.n_slices;
    H.n_slices_hi = (uint32_t)(P.n_slices >> 32);
    H.off_col = (uint32_t)img.size();
    for (int j = 0; j < w.pe; ++j) {
        std::vector<uint32_t> col(W, 0);
        for (int f = 0; f < F; ++f)
            if (used[f].mask >> j & 1) col[f / 32] |= 1u << (f % 32);
        img.insert(img.end(), col.begin(), col.end());
    }
    H.off_cvec = (uint32_t)img.size();
    {
        std::vector<uint32_t> cv(W, 0);
        for (int f = 0; f < F; ++f)
            if (used[f].cst) cv[f / 32] |= 1u << (f % 32);
        for (int k = 0; k < W; ++k) cv[k] ^= zflip[k];
        img.insert(img.end(), cv.begin(), cv.end());
    }
    H.off_zmask = (uint32_t)img.size();
    img.insert(img.end(), zmask.begin(), zmask.end());
    // a pattern no block can match: the masked start vector of a surviving term is one of the
    // 2^KB combinations of the inner columns on the vanishing bits, all inside zmask
    H.off_never = (uint32_t)img.size();
    {
        std::vector<uint32_t> nv(W, 0);
        bool outside = false;
        for (int k = 0; k < W; ++k) {
            nv[k] = ~zmask[k];
            outside = outside || nv[k] != 0;
        }
        if (!outside && g >= KB) {
            std::vector<std::vector<uint32_t>> combos;
            for (int y = 0; y < KS; ++y) {
                std::vector<uint32_t> c(W, 0);
                for (int j = 0; j < KB; ++j)
                    if (y >> j & 1)
                        for (int f = 0; f < F; ++f)
                            if (used[f].mask >> j & 1) c[f / 32] ^= 1u << (f % 32);
                for (int k = 0; k < W; ++k) c[k] &= zmask[k];
                combos.push_back(c);
            }
            for (uint32_t cand = 1;; ++cand) {
                std::vector<uint32_t> c(W, 0);
                c[0] = cand;
                if (std::find(combos.begin(), combos.end(), c) == combos.end()) {
                    nv = c;
                    break;
                }
            }
        }
        img.insert(img.end(), nv.begin(), nv.end());
    }
    // The masked start vector a of a block has a surviving term at step k iff a equals the
    // combination of the inner columns on the vanishing bits picked by gray(k).  A reduced
    // basis of their span (each basis vector owns a pivot bit no other has) lets a lane read the
    // coordinates of a off its pivot bits: a is in the span iff it equals that combination, and
    // the inner columns' coefficients of a basis vector turn the coordinates into gray(k); the
    // null space (dependent columns) gives the other steps with the same vector.
    {
        std::vector<std::vector<uint32_t>> basis;  // reduced basis vectors
        std::vector<int> pivot;                    // their pivot bits
        std::vector<uint32_t> comb;                // inner columns making up each
        std::vector<uint32_t> kern;                // null-space basis (KB-bit combinations)
        if (g >= KB) {
            for (int j = 0; j < KB; ++j) {
                std::vector<uint32_t> v(W, 0);
                for (int f = 0; f < F; ++f)
                    if (used[f].mask >> j & 1) v[f / 32] |= 1u << (f % 32);
                for (int k = 0; k < W; ++k) v[k] &= zmask[k];
                uint32_t c = 1u << j;
                for (size_t i = 0; i < basis.size(); ++i)
                    if (v[pivot[i] / 32] >> (pivot[i] % 32) & 1) {
                        for (int k = 0; k < W; ++k) v[k] ^= basis[i][k];
                        c ^= comb[i];
                    }
                int pb = -1;
                for (int k = 0; k < W && pb < 0; ++k)
                    if (v[k]) pb = 32 * k + __builtin_ctz(v[k]);
                if (pb < 0) {
                    kern.push_back(c);
                    continue;
                }
                for (size_t i = 0; i < basis.size(); ++i)
                    if (basis[i][pb / 32] >> (pb % 32) & 1) {
                        for (int k = 0; k < W; ++k) basis[i][k] ^= v[k];
                        comb[i] ^= c;
                    }
                basis.push_back(v);
                pivot.push_back(pb);
                comb.push_back(c);
            }
        }
        H.inner_rank = (uint32_t)basis.size();
        H.off_ibasis = (uint32_t)img.size();
        for (size_t i = 0; i < basis.size(); ++i) {
            img.push_back((uint32_t)(pivot[i] / 32));
            img.push_back((uint32_t)(pivot[i] % 32));
            img.push_back(comb[i]);
            img.insert(img.end(), basis[i].begin(), basis[i].end());
        }
        // padded to KB entries with zero entries (they change nothing), so the kernel reads all
        // of them at once without testing the rank
        for (size_t i = basis.size(); i < (size_t)KB; ++i) img.insert(img.end(), 3 + W, 0u);
        H.off_ikern = (uint32_t)img.size();
        img.insert(img.end(), kern.begin(), kern.end());
    }
    H.off_slots = (uint32_t)img.size();
    for (int s = 0; s < N_STATS; ++s)
        H.stat_base[s] = (int32_t)(s == STAT_R ? mod8(base[s]) : base[s]);
    if (use_ntab) {
        // the table carries the node factors; the phase slots count the linear terms alone
        for (int s = 0; s < N_STATS; ++s) {
            std::fill(wt[s].begin(), wt[s].end(), 0LL);
            H.stat_base[s] = 0;
        }
        wt[STAT_R] = wt_lin;
        for (int b = 0; b < ntab_bits; ++b) {
            wt_tab[b] = wt_lin[b];
            wt[STAT_R][b] = 0;
        }
        H.stat_base[STAT_R] = (int32_t)mod8(base_lin);
    }
    int active_slots = 0;
    uint32_t active_mask = 0;
    for (int i = 0; i < kSlots; ++i) {
        const int s = slot_stat(i), wgt = slot_weight(i);
        std::vector<uint32_t> mask(W, 0);
        bool any = false;
        for (int f = 0; f < F; ++f) {
            long long v = wt[s][f];
            bool on;
            if (s == STAT_R) on = (mod8(v) & wgt) != 0;
            else on = v == wgt;
            if (on) {
                mask[f / 32] |= 1u << (f % 32);
                any = true;
            }
        }
        for (int f = 0; f < F; ++f) {
            long long v = wt[s][f];
            if (s != STAT_R && v != 0 && v != 1 && v != -1 && !(s == STAT_E && (v == 2 || v == -2))) {
                *err = "internal: statistic weight outside the fixed slots";
                return SIM_EINVAL;
            }
        }
        img.push_back(any ? (uint32_t)(int32_t)wgt : 0u);
        img.insert(img.end(), mask.begin(), mask.end());
        active_slots += any ? 1 : 0;
        if (any) active_mask |= 1u << i;
    }
    if (use_ntab && (active_mask & ~slot_set_of(3u) & kSlotSetAll)) {
        *err = "internal: a weight-4 phase slot beside the node table";
        return SIM_EINVAL;
    }
    H.slot_menu = use_ntab ? 3u
                : (active_mask & ~kSlotSetPhase) == 0 ? 2u
                : (active_mask & ~kSlotSetNodes) == 0 ? 1u : 0u;
    {
        // node-factor bits are allocated first, then the combined weight-4 phase term, so with
        // at most 31 node factors the A, B, E and R*4 masks live in word 0
        bool word0 = W > 1;
        for (int i = 0; i < kSlots && word0; ++i) {
            if (slot_stat(i) == STAT_R && slot_weight(i) != 4) continue;
            const uint32_t *m = img.data() + H.off_slots + i * (W + 1) + 1;
            for (int k = 1; k < W; ++k) word0 = word0 && m[k] == 0;
        }
        H.node_word0 = word0 ? 1u : 0u;
    }
    // a term's coordinates are at most 2^(node factors), a lane's block holds 2^KB terms
    H.block_sum32 = acc_mode == ACC_I64 && n_nodes + KB <= 30 ? 1u : 0u;
    active_slots = __builtin_popcount(slot_set_of(H.slot_menu) & kSlotSetAll);
    // monomials in packed positions
    const uint64_t walk_mask = g >= 64 ? ~0ull : (((uint64_t)1 << g) - 1);
    std::vector<std::pair<int, uint64_t>> monos;
    for (const auto &m : w.mono) {
        uint64_t pm = 0;
        for (int v : m.first) pm |= (uint64_t)1 << pos_of[v];
        monos.push_back({m.second, pm});
    }
    H.off_monohi = (uint32_t)img.size();
    for (const auto &m : monos) {
        if (m.second & walk_mask) continue;
        uint64_t hm = m.second >> g;
        img.push_back((uint32_t)m.first);
        img.push_back((uint32_t)hm);
        img.push_back((uint32_t)(hm >> 32));
        H.n_monohi++;
    }
    // per walk position i: always-firing entries (uniform sum, or per-lane list) and the
    // entries that depend on walk bits above i; entries needing a bit below i - 1 never fire
    std::vector<int> ui(g, 0);
    std::vector<std::vector<uint32_t>> al(g), per(g);
    for (int i = 0; i < g; ++i) {
        for (const auto &m : monos) {
            if (!(m.second >> i & 1)) continue;
            const uint64_t others = m.second & ~((uint64_t)1 << i);
            const uint32_t wm = (uint32_t)(others & walk_mask);
            const uint64_t hm = others >> g;
            const uint32_t below = i > 0 ? (uint32_t)(((uint64_t)1 << (i - 1)) - 1) : 0u;
            if (wm & below) continue;                        // needs a bit that is 0: never fires
            const uint32_t above = wm >> (i + 1) << (i + 1);  // bits above i decide
            if (!above) {
                if (!hm) ui[i] = mod8(ui[i] + m.first);
                else {
                    al[i].push_back((uint32_t)m.first);
                    al[i].push_back((uint32_t)hm);
                    al[i].push_back((uint32_t)(hm >> 32));
                }
            } else {
                per[i].push_back((uint32_t)m.first);
                per[i].push_back(above);
                per[i].push_back((uint32_t)hm);
                per[i].push_back((uint32_t)(hm >> 32));
            }
        }
    }
    H.off_ui = (uint32_t)img.size();
    for (int i = 0; i < g; ++i) img.push_back((uint32_t)ui[i]);
    H.off_aidx = (uint32_t)img.size();
    uint32_t acc = 0;
    for (int i = 0; i <= g; ++i) {
        img.push_back(acc);
        if (i < g) acc += (uint32_t)(al[i].size() / 3);
    }
    H.off_al = (uint32_t)img.size();
    for (int i = 0; i < g; ++i) img.insert(img.end(), al[i].begin(), al[i].end());
    H.off_didx = (uint32_t)img.size();
    acc = 0;
    for (int i = 0; i <= g; ++i) {
        img.push_back(acc);
        if (i < g) acc += (uint32_t)(per[i].size() / 4);
    }
    while (img.size() % 4) img.push_back(0);  // entries are read as one 16-byte load
    H.off_delta = (uint32_t)img.size();
    for (int i = 0; i < g; ++i) img.insert(img.end(), per[i].begin(), per[i].end());

    // inner-block phase vectors (walks of at least KB positions): for each monomial with an
    // inner variable, field k of the (even, odd) vector is c * ([inner part set at step k] -
    // [... at step 0]) mod 8; grouped by what else the monomial needs
    const int C3S = 4 * NF;  // words per inner-vector entry of a flip (aligned, one load)
    std::vector<uint32_t> inner_vec(2 * NF, 0);
    std::vector<uint32_t> c2, c3all;
    std::vector<std::vector<uint32_t>> c3pos(g);  // per outer walk position
    if (g >= KB) {
        const uint64_t inner_mask = ((uint64_t)1 << KB) - 1;
        auto field_add = [](uint32_t a, uint32_t b) { return (a + b) & 0x77777777u; };
        for (const auto &m : monos) {
            const uint64_t I = m.second & inner_mask;
            if (!I) continue;
            std::vector<uint32_t> vec(2 * NF, 0);  // even[NF], odd[NF]
            for (int odd = 0; odd < 2; ++odd) {
                const uint64_t y0 = (uint64_t)odd << (KB - 1);
                const int f0 = (I & y0) == I;
                for (int k = 1; k < KS; ++k) {
                    const uint64_t y = (uint64_t)(k ^ (k >> 1)) ^ y0;
                    const int f = (I & y) == I;
                    vec[odd * NF + k / 8] |= (uint32_t)mod8((long long)m.first * (f - f0)) << (4 * (k % 8));
                }
            }
            const uint32_t om = (uint32_t)(m.second & walk_mask & ~inner_mask);
            const uint64_t hm = m.second >> g;
            if (!om && !hm) {
                for (int k = 0; k < 2 * NF; ++k) inner_vec[k] = field_add(inner_vec[k], vec[k]);
                continue;
            }
            if (!om) {
                c2.insert(c2.end(), vec.begin(), vec.end());
                c2.push_back((uint32_t)hm);
                c2.push_back((uint32_t)(hm >> 32));
                continue;
            }
            c3all.insert(c3all.end(), vec.begin(), vec.end());
            c3all.push_back(om);
            c3all.push_back((uint32_t)hm);
            c3all.push_back((uint32_t)(hm >> 32));
            // needs outer walk bits: its activation toggles when one of them flips while the
            // others are set; at a flip of outer position i the outer bits below i - 1 are clear
            for (int i = KB; i < g; ++i) {
                if (!(om >> i & 1)) continue;
                const uint32_t other = om & ~(1u << i);
                const uint32_t clear_below = i - 1 > KB ? ((1u << (i - 1)) - 1) & ~((1u << KB) - 1) : 0u;
                if (other & clear_below) continue;
                std::vector<uint32_t> &dst = c3pos[i];
                dst.insert(dst.end(), vec.begin(), vec.end());
                dst.push_back(other);
                dst.push_back((uint32_t)hm);
                dst.push_back((uint32_t)(hm >> 32));
                while (dst.size() % C3S) dst.push_back(0);
            }
        }
    }
    H.off_inner = (uint32_t)img.size();
    img.insert(img.end(), inner_vec.begin(), inner_vec.end());
    H.off_c2 = (uint32_t)img.size();
    H.n_c2 = (uint32_t)(c2.size() / (2 * NF + 2));
    img.insert(img.end(), c2.begin(), c2.end());
    H.off_c3idx = (uint32_t)img.size();
    std::vector<uint32_t> c3start(g + 1, 0);
    {
        uint32_t n = 0;
        for (int i = 0; i <= g; ++i) {
            img.push_back(n);
            c3start[i] = n;
            if (i < g) n += (uint32_t)(c3pos[i].size() / C3S);
        }
        H.n_c3 = n;
    }
    while (img.size() % 8) img.push_back(0);  // entries are read with 32-byte loads
    H.off_c3 = (uint32_t)img.size();
    for (int i = 0; i < g; ++i) img.insert(img.end(), c3pos[i].begin(), c3pos[i].end());
    // one record per walk position: everything a flip of it reads first (entry ranges as
    // 16-bit halves)
    if (img[H.off_didx + g] > 0xFFFFu || c3start[g] > 0xFFFFu) {
        *err = "more than 65535 walk list entries";
        return SIM_ERANGE;
    }
    while (img.size() % 4) img.push_back(0);
    H.off_pos = (uint32_t)img.size();
    for (int i = 0; i < g; ++i) {
        const uint32_t *didx = img.data() + H.off_didx;
        const uint32_t rec[4] = {(uint32_t)ui[i], didx[i] | (didx[i + 1] << 16), c3start[i] | (c3start[i + 1] << 16),
                                 gcol[i]};
        img.insert(img.end(), rec, rec + 4);
    }
    // for a walk that starts inside a slice: each inner-and-outer monomial once, with its whole
    // outer mask, and every monomial with a walk part (c, walk mask, slice mask lo, hi)
    H.off_c3all = (uint32_t)img.size();
    H.n_c3all = (uint32_t)(c3all.size() / (2 * NF + 3));
    img.insert(img.end(), c3all.begin(), c3all.end());
    H.off_monowalk = (uint32_t)img.size();
    for (const auto &m : monos) {
        const uint32_t wm = (uint32_t)(m.second & walk_mask);
        if (!wm) continue;
        const uint64_t hm = m.second >> g;
        img.push_back((uint32_t)m.first);
        img.push_back(wm);
        img.push_back((uint32_t)hm);
        img.push_back((uint32_t)(hm >> 32));
        H.n_monowalk++;
    }

    // form monomials: 8 words each (c | deg << 8 | j1 << 16 | j2 << 24, j3, and the three
    // forms' lambda as lo, hi words; lambda holds the block's 2^KB steps, KB <= 6); the forms:
    // 4 words each (slice mask lo, hi, constant, 0)
    H.block_flush128 = flush128 ? 1u : 0u;
    // small programs whose monomials are all form monomials (no per-slice walk lists): two
    // waves per unit, each evaluating half of every 64-term block
    H.term_split = (fm_only && KB == 6 && g >= KB && !has_zero) ? 2u : 1u;
    H.n_fmono = (uint32_t)fmono.size();
    H.n_mforms = (uint32_t)mforms.size();
    H.gcol_top = g >= KB && KB > 0 ? gcol[KB - 1] : 0u;
    while (img.size() % 8) img.push_back(0);
    H.off_fmono = (uint32_t)img.size();
    {
        auto lambda = [&](const IrForm &f) {
            uint64_t lam = 0;
            if (g >= KB)
                for (int k = 0; k < KS; ++k) {
                    const uint64_t y = (uint64_t)(k ^ (k >> 1));
                    if (__builtin_popcountll(f.mask & y & (((uint64_t)1 << KB) - 1)) & 1) lam |= (uint64_t)1 << k;
                }
            return lam;
        };
        for (size_t e = 0; e < fmono.size(); ++e) {
            const auto &ix = fm_idx[e];
            const int deg = ix[2] >= 0 ? 3 : 2;
            uint32_t ent[8] = {0, 0, 0, 0, 0, 0, 0, 0};
            ent[0] = (uint32_t)mod8(fmono[e].c) | ((uint32_t)deg << 8) | ((uint32_t)ix[0] << 16) | ((uint32_t)ix[1] << 24);
            ent[1] = deg == 3 ? (uint32_t)ix[2] : 0u;
            for (int t = 0; t < deg; ++t) {
                const uint64_t lam = lambda(mforms[ix[t]]);
                ent[2 + 2 * t] = (uint32_t)lam;
                ent[3 + 2 * t] = (uint32_t)(lam >> 32);
            }
            img.insert(img.end(), ent, ent + 8);
        }
    }
    // group boundaries: 15 words, group k = (three forms: k >= 7, coefficient k % 7 + 1) holds
    // entries [grp[k], grp[k + 1])
    H.off_fmgrp = (uint32_t)img.size();
    {
        uint32_t at = 0;
        for (int d3 = 0; d3 < 2; ++d3)
            for (int c = 1; c < 8; ++c) {
                img.push_back(at);
                for (size_t e = 0; e < fmono.size(); ++e)
                    if ((fm_idx[e][2] >= 0) == (d3 == 1) && mod8(fmono[e].c) == c) ++at;
            }
        img.push_back(at);
    }
    // teams of two waves: per half (steps 32h .. 32h + 31 of a block) a table of the entries
    // with that half's pattern words only and the form indices as whole words (no field
    // extraction or selection on the scalar unit).  Each group is padded with null entries
    // (pattern m & ~m = 0) to whole batches of the kernel's loop (8 two-form entries, 4
    // three-form entries), so that no group ends in single loads.  At off_fmh: 16 words of
    // padded bounds (two-form groups 0..6 in d2[0..7], three-form groups in d3[0..7]), then
    // the two half tables fmh_stride words apart: two-form entries of 4 words (j1, j2, lambda1,
    // lambda2), then at fmh_off3 three-form entries of 8 words (j1, j2, j3, lambda1..3, 0, 0).
    H.off_fmh = H.fmh_stride = H.fmh_off3 = 0;
    if (H.term_split == 2 && !fmono.empty()) {
        while (img.size() % 8) img.push_back(0);
        const uint32_t *grp = img.data() + H.off_fmgrp;
        uint32_t d2[8], d3[8];
        std::vector<int> src2, src3;  // entry of the main table, -1 for a null entry
        d2[0] = d3[0] = 0;
        for (int k = 0; k < 7; ++k) {
            for (uint32_t e = grp[k]; e < grp[k + 1]; ++e) src2.push_back((int)e);
            while (src2.size() % 8) src2.push_back(-1);
            d2[k + 1] = (uint32_t)src2.size();
            for (uint32_t e = grp[7 + k]; e < grp[8 + k]; ++e) src3.push_back((int)e);
            while (src3.size() % 4) src3.push_back(-1);
            d3[k + 1] = (uint32_t)src3.size();
        }
        H.off_fmh = (uint32_t)img.size();
        img.insert(img.end(), d2, d2 + 8);
        img.insert(img.end(), d3, d3 + 8);
        H.fmh_off3 = 4 * (uint32_t)src2.size();  // a multiple of 32 words
        H.fmh_stride = H.fmh_off3 + 8 * (uint32_t)src3.size();
        for (int h = 0; h < 2; ++h) {
            const size_t base = img.size();
            img.resize(base + H.fmh_stride, 0u);
            for (size_t i = 0; i < src2.size(); ++i) {
                uint32_t *dst = img.data() + base + 4 * i;
                if (src2[i] < 0) {
                    dst[3] = 0xFFFFFFFFu;  // j1 = j2 = 0, lambda1 = 0, lambda2 = ~0
                    continue;
                }
                const uint32_t *src = img.data() + H.off_fmono + 8 * src2[i];
                dst[0] = (src[0] >> 16) & 0xFFu;
                dst[1] = src[0] >> 24;
                dst[2] = src[2 + h];
                dst[3] = src[4 + h];
            }
            for (size_t i = 0; i < src3.size(); ++i) {
                uint32_t *dst = img.data() + base + H.fmh_off3 + 8 * i;
                if (src3[i] < 0) {
                    dst[4] = 0xFFFFFFFFu;  // j1 = j2 = j3 = 0, lambda2 = ~0, the others 0
                    continue;
                }
                const uint32_t *src = img.data() + H.off_fmono + 8 * src3[i];
                dst[0] = (src[0] >> 16) & 0xFFu;
                dst[1] = src[0] >> 24;
                dst[2] = src[1];
                dst[3] = src[2 + h];
                dst[4] = src[4 + h];
                dst[5] = src[6 + h];
            }
        }
    }
    H.off_mforms = (uint32_t)img.size();
    for (const auto &f : mforms) {
        const uint64_t hm = g >= 64 ? 0 : f.mask >> g;
        img.push_back((uint32_t)hm);
        img.push_back((uint32_t)(hm >> 32));
        img.push_back((uint32_t)f.cst);
        img.push_back(0u);
    }
    H.off_gcol = (uint32_t)img.size();
    img.insert(img.end(), gcol.begin(), gcol.end());
    H.off_scol = (uint32_t)img.size();
    H.fm_s0 = 0;
    for (size_t j = 0; j < mforms.size(); ++j)
        if (mforms[j].cst) H.fm_s0 |= 1u << j;
    for (int i = g; i < w.pe; ++i) {
        uint32_t c = 0;
        for (size_t j = 0; j < mforms.size(); ++j)
            if (mforms[j].mask >> i & 1) c |= 1u << j;
        img.push_back(c);
    }

    // ---- value table
    H.d_off = (int32_t)(-dmin);
    H.table_n = (uint32_t)(nd * 16 + 1);
    H.zero_entry = (uint32_t)(nd * 16);
    H.acc = acc_mode;
    H.q_limbs = q_limbs;
    {
        const size_t base_lds = acc_mode == ACC_CLASS ? (size_t)H.zero_entry * q_limbs * 8 : (size_t)H.table_n * 32;
        H.ntab_lds = (uint32_t)((base_lds + 15) & ~(size_t)15);
    }
    // the node table: entry u describes the node factors with bits u of L
    H.off_ntab = (uint32_t)img.size();
    if (use_ntab) {
        H.ntab_n = 1u << ntab_bits;
        for (uint32_t u = 0; u < H.ntab_n; ++u) {
            long long st[N_STATS] = {0, 0, 0, 0};
            bool vanish = false;
            for (int j = 0; j < n_nodes; ++j) {
                const int bit = (int)(u >> j & 1) ^ (int)(zflip[0] >> j & 1);
                const int v = bit ? w.nodes[j].second.second : w.nodes[j].second.first;
                if (v == 4) vanish = true;
                for (int s2 = 0; s2 < N_STATS; ++s2) st[s2] += fns[s2](v);
            }
            for (int b = 0; b < ntab_bits; ++b)  // linear weights count the bits of L as stored
                if (u >> b & 1) st[STAT_R] += wt_tab[b];
            uint32_t e = 1u;
            if (!vanish) {
                const long long m = std::min(st[STAT_A], st[STAT_B]);
                const long long dd = st[STAT_A] - st[STAT_B] - dmin;
                const long long ee = st[STAT_E] + m;
                const long long rr = mod8(st[STAT_R] + 2 * m);
                e = ((uint32_t)dd << 1) | ((uint32_t)ee << 8) | ((uint32_t)rr << 16);
            }
            img.push_back(e);
        }
    }
    // Surviving steps of a block by the vanishing bits, when those all lie in word 0 (compacting
    // walks): step k of a block survives iff P(gray(k)) & zmask = a, a = L & zmask at the block's
    // first term, P(y) the XOR of the inner columns picked by y.  The at most 2^KB keys
    // P(gray(k)) & zmask, each with the mask of its steps, go to a hashed table of
    // ztab_slots_for(KB)
    // (key, mask) pairs; the multiplier is the first of a fixed sequence that maps the keys to
    // distinct slots.  Then come the KS values P(gray(k)) (W words each).  Both are copied to
    // LDS after the other tables.
    H.ztab_bits = 0;
    H.ztab_mult = 0;
    H.off_ztab = (uint32_t)img.size();
    const uint32_t zslots = ztab_slots_for(KB);
    H.ztab_shift = 32u - (uint32_t)__builtin_ctz(zslots);
    {
        const size_t end_lds = H.ntab_n ? (size_t)H.ntab_lds + (size_t)H.ntab_n * 4
                                        : (acc_mode == ACC_CLASS ? (size_t)H.zero_entry * q_limbs * 8
                                                                 : (size_t)H.table_n * 32);
        H.ztab_lds = (uint32_t)((end_lds + 15) & ~(size_t)15);
        bool word0 = has_zero && g >= KB && W <= 4 && zmask[0] != 0;
        for (int k = 1; k < W; ++k) word0 = word0 && zmask[k] == 0;
        if (word0) {
            std::vector<uint32_t> pstep((size_t)KS * W, 0);
            for (int k = 0; k < KS; ++k) {
                const int y = k ^ (k >> 1);
                for (int j = 0; j < KB; ++j)
                    if (y >> j & 1)
                        for (int w2 = 0; w2 < W; ++w2) pstep[(size_t)k * W + w2] ^= img[H.off_col + j * W + w2];
            }
            std::map<uint32_t, uint64_t> steps;  // key -> mask of its steps
            for (int k = 0; k < KS; ++k) steps[pstep[(size_t)k * W] & zmask[0]] |= (uint64_t)1 << k;
            uint64_t state = 0x243F6A8885A308D3ull;  // a fixed sequence of odd multipliers
            for (int attempt = 0; attempt < 4096 && !H.ztab_mult; ++attempt) {
                state += 0x9E3779B97F4A7C15ull;
                uint64_t x = state;
                x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
                x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
                const uint32_t mult = (uint32_t)(x ^ (x >> 31)) | 1u;
                std::vector<char> used_slot(zslots, 0);
                bool ok = true;
                for (const auto &kv : steps) {
                    const uint32_t slot = (kv.first * mult) >> H.ztab_shift;
                    if (used_slot[slot]) {
                        ok = false;
                        break;
                    }
                    used_slot[slot] = 1;
                }
                if (ok) H.ztab_mult = mult;
            }
            if (H.ztab_mult) {
                H.ztab_bits = (uint32_t)__builtin_popcount(zmask[0]);
                std::vector<uint32_t> zt(4 * zslots, 0);  // (key, mask lo, hi, 0); empty slots have mask 0
                for (const auto &kv : steps) {
                    const uint32_t slot = (kv.first * H.ztab_mult) >> H.ztab_shift;
                    zt[4 * slot] = kv.first;
                    zt[4 * slot + 1] = (uint32_t)kv.second;
                    zt[4 * slot + 2] = (uint32_t)(kv.second >> 32);
                }
                img.insert(img.end(), zt.begin(), zt.end());
                img.insert(img.end(), pstep.begin(), pstep.end());
            }
        }
        // the half tables of the form monomials (two-wave teams) follow every other LDS table;
        // when they would not fit the kernels' dynamic LDS, the program is evaluated whole
        // blocks per wave instead (the form monomials read from the image)
        H.fmh_lds = 0;
        if (H.off_fmh) {
            const size_t end_z = H.ztab_bits ? (size_t)H.ztab_lds + (4 * (size_t)zslots + (size_t)KS * W) * 4 : end_lds;
            const size_t at = (end_z + 15) & ~(size_t)15;
            if (at + (16 + 2 * (size_t)H.fmh_stride) * 4 <= kMaxDynLdsBytes) {
                H.fmh_lds = (uint32_t)at;
            } else {
                H.term_split = 1;
                H.off_fmh = H.fmh_stride = H.fmh_off3 = 0;
            }
        }
    }
    std::vector<int64_t> table((size_t)H.table_n * 4, 0);
    for (int d = (int)dmin; d <= (int)dmax; ++d)
        for (int r = 0; r < 8; ++r)
            for (int e = 0; e < 2; ++e) {
                Zw z = table_value(d, r, e);
                size_t idx = ((size_t)(d - dmin) * 8 + r) * 2 + e;
                for (int k = 0; k < 4; ++k) {
                    if (z.c[k] > (i128)INT64_MAX || z.c[k] < (i128)INT64_MIN) {
                        *err = "table entry exceeds int64";
                        return SIM_ERANGE;
                    }
                    table[idx * 4 + k] = (int64_t)z.c[k];
                }
            }
    size_t word_bytes = img.size() * 4;
    size_t tab_off = (word_bytes + 7) & ~(size_t)7;
    H.table_byte_off = (uint32_t)tab_off;
    H.image_bytes = (uint32_t)(tab_off + table.size() * 8);
    P.blob.assign(H.image_bytes, 0);
    if (!img.empty()) memcpy(P.blob.data(), img.data(), word_bytes);
    memcpy(P.blob.data() + tab_off, table.data(), table.size() * 8);

    // ---- algorithmic work per term, in int32 lane (vector) operations counted from the packed
    // program; work on wave-uniform values (list walking, program constants) runs on the
    // scalar unit and is not counted.  The statistics of a term, needed only where no factor
    // vanishes (an exact fraction: the vanishing conditions are affine in x): per mask one AND
    // and one popcount-accumulate per word it spans (with the node table: one AND and one LDS
    // read for all node factors), the table index and shift (8), the accumulation (int64 12,
    // int128 40, class counter 5) and with monomials the term's phase field (2).
    //  * walks of at least KB positions: with factors that can vanish and W <= 4 the vanishing
    //    test is per block (below) and a surviving term costs the rebuild of its form vector
    //    (W); with wider form vectors each term's vanishing test (a W-word compare) as well;
    //    otherwise each term's column XOR (W).  Per block: the outer column XOR (W), with
    //    vanishing factors the block's test and the end XOR (the table of surviving steps:
    //    mask, hash product and shift, key compare and the end XOR, 4 + W; the reduced basis:
    //    KB bit extracts with W XORs each, the compare and the end XOR, KB (2 + W) + 2W), with
    //    monomials
    //    the vector-pair selection (NF), the flip's own change (5), 5 per firing slice-dependent
    //    flip entry and 4 + 4 NF per toggling inner-vector entry (slice test, 2 NF field adds);
    //  * shorter walks: per term the column XOR (W), the vanishing test (2W) and the flip
    //    (5 plus 5 per firing slice-dependent entry);
    //  * per slice: the high parameters into L (2W each), 5 per slice-dependent monomial entry,
    //    4 per walk position for the packed always-firing fields, 4 + 4 NF per inner-vector entry,
    //    2 per slice bit for the form monomials' forms (S);
    //  * form monomials, per block: O (1); per monomial a bit extract and KW XORs per form (KW =
    //    words of a block's 2^KB-bit pattern), KW ANDs per further form, and the add of c times the
    //    pattern to three bit planes (5, 3, 1 KW for the bits of c); the planes to 4-bit fields (23
    //    per field word) and their add (2 per field word).  Shorter walks: per term O (1) and 5 per
    //    monomial.  Blocks moved from int64 to int128 sums: 16 per block.
    {
        const double nz = nonzero_fraction(used, w.nodes);
        P.nonzero_fraction = nz;
        const bool mono = any_mono;
        const bool blocks = g >= KB;
        const bool compact = blocks && has_zero && W <= 4;
        // the slot set of the kernel variant the program is dispatched to (int128 mode: all)
        const bool nw0_kernel = H.acc != ACC_I128 && W > 1 && W < 16 && H.node_word0 && H.slot_menu <= 1;
        const uint32_t set = H.acc == ACC_I128 ? kSlotSetAll
                                               : slot_set_of(H.slot_menu) | (nw0_kernel ? kSlotsNodeWord0 : 0u);
        // node-table and node-word-0 programs in int64 mode whose block sums fit in 32 bits,
        // walking blocks without compaction, add a block's terms in 32 bits (one shift-and-add
        // per coordinate) and move them to int64 per block
        const bool b32 = H.acc == ACC_I64 && H.block_sum32 && (H.slot_menu == 3 || nw0_kernel) && blocks && !compact;
        const double acc_ops = b32 ? 4.0 : H.acc == ACC_I64 ? 12.0 : H.acc == ACC_I128 ? 40.0 : 5.0;
        const double flush_ops = b32 ? 12.0 / KS : 0.0;
        double slot_ops = 0;
        for (int i = 0; i < kSlots; ++i)
            if (set >> i & 1) slot_ops += 2.0 * slot_words(set, i, W);
        const double stats = 8 + acc_ops + slot_ops + (mono ? 2 : 0);
        double ops;
        if (compact) ops = nz * (W + stats);
        else if (blocks && has_zero) ops = W + flush_ops + nz * (W + stats);
        else if (blocks) ops = W + flush_ops + stats;
        else ops = W + (has_zero ? 2.0 * W : 0) + nz * stats;
        double setup = (double)(w.pe - g) * 2.0 * W;
        if (mono) setup += 5.0 * H.n_monohi + 5.0 * img[H.off_aidx + g] + 4.0 * g + (blocks ? (4.0 + 4.0 * NF) * H.n_c2 : 0);
        const uint64_t steps = (uint64_t)1 << g;
        double walk = 0;
        const uint32_t *didx = img.data() + H.off_didx;
        const uint32_t *de = img.data() + H.off_delta;
        auto flip_cost = [&](int i, uint32_t gray) {
            double c = 0;
            if (!mono) return c;
            c += 5;
            for (uint32_t e = didx[i]; e < didx[i + 1]; ++e) {
                const uint32_t wm = de[4 * e + 1];
                const bool hi = de[4 * e + 2] || de[4 * e + 3];
                if ((gray & wm) == wm && hi) c += 5;
            }
            return c;
        };
        if (!blocks) {
            for (uint64_t t = 1; t < steps; ++t)
                walk += flip_cost(__builtin_ctzll(t), (uint32_t)(t ^ (t >> 1)));
        } else {
            const uint64_t nb = steps >> KB;
            const uint32_t *c3idx = img.data() + H.off_c3idx;
            const uint32_t *c3 = img.data() + H.off_c3;
            const double vanish_test = !compact ? 2.0 * W : H.ztab_bits ? 4.0 + W : KB * (2.0 + W) + 2.0 * W;
            walk += (double)nb * ((has_zero ? vanish_test : 0) + (mono ? NF : 0));
            for (uint64_t b = 1; b < nb; ++b) {
                const int i = KB + __builtin_ctzll(b);
                const uint32_t gray = (uint32_t)((b ^ (b >> 1)) << KB);
                walk += W + flip_cost(i, gray);
                if (!mono) continue;
                for (uint32_t e = c3idx[i]; e < c3idx[i + 1]; ++e) {
                    const uint32_t other = c3[C3S * e + 2 * NF];
                    if ((gray & other) == other) walk += 4 + 4 * NF;
                }
            }
        }
        const double KW = KS >= 32 ? KS / 32.0 : 1.0;
        double fm_block = 0;
        if (!fmono.empty()) {
            fm_block = 1 + NF * (23.0 + 2.0);
            for (size_t e = 0; e < fmono.size(); ++e) {
                const int deg = fm_idx[e][2] >= 0 ? 3 : 2;
                const int c = mod8(fmono[e].c);
                fm_block += deg * (1 + KW) + (deg - 1) * KW + ((c & 1) ? 5 : 0) * KW + ((c & 2) ? 3 : 0) * KW +
                            ((c & 4) ? 1 : 0) * KW;
            }
            setup += 2.0 * (w.pe - g);  // S: one masked column XOR per slice bit
        }
        if (blocks && H.term_split == 2) {
            // both waves of a team extract the forms' bits; each takes one pattern word
            for (size_t e = 0; e < fmono.size(); ++e) fm_block += (fm_idx[e][2] >= 0 ? 3 : 2);
            fm_block += 2.0 * W;  // the second half's start state
        }
        if (blocks) walk += (double)(steps >> KB) * (fm_block + (flush128 ? 16.0 : 0.0));
        else if (!fmono.empty()) ops += 1 + 5.0 * fmono.size();
        P.ops_per_term = ops + (setup + walk) / (double)steps;
    }

    P.c0 = w.c0;
    P.e = w.e;
    P.zero = w.zero;
    zw_canonicalise(&P.c0, &P.e);
    return SIM_OK;
}
