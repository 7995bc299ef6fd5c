// Host-side compiler: Clifford+T circuit and query -> term program.
//
// 1. Diagram.  The circuit is closed with |0^n> and the query's effect (Section 2.2) and
//    written as a graph-like ZX diagram (Section 2.1): Z spiders joined by Hadamard edges.
//    Its scalar is, exactly,
//        scalar * sum_{z in {0,1}^V} w^{ sum_v (a_v + 4 l_v(x)) z_v + 4 sum_{uv in E} z_u z_v },
//    one Boolean z_v per spider, a_v its phase in units of pi/4, and l_v(x) a parity of the
//    Boolean parameters x (the polar phase alpha + pi (p1 xor ... xor pn) of Eq. 1).
//    Each wire carries a parity of spiders: H starts a new spider joined to that parity
//    (scalar 1/sqrt2), CNOT adds parities, a Z-phase gate adds its phase to the parity it acts
//    on (equal parities fuse, as spider fusion does), and an effect <y| is a new spider joined
//    to the wire's parity with phase pi*y (scalar 1/2).  A phase on a parity of several
//    spiders becomes, if it is a multiple of pi/2, phases and edges on those spiders, and
//    otherwise a phase gadget (hub and leaf spider, scalar 1/2).
// 2. Parametric Clifford simplification (the polar rules of Section 3.1 and Appendix B; every
//    phase stays fixed or polarised, Lemma 2): local complementation removes +-pi/2 spiders,
//    pivoting removes pairs of adjacent 0/pi spiders, a 0/pi spider with one neighbour fixes
//    that neighbour to an affine function of x, a 0/pi spider with two neighbours fuses them,
//    and an isolated spider leaves the factor 1 + e^{i(alpha + pi l(x))} (the node subterm
//    of the Appendix C table).  Phases products of two polar phases (the pi-pair subterm) are
//    written with 4 l1 l2 = 2 l1 + 2 l2 - 2 (l1 xor l2) (mod 8), and half-pi terms as 2 l.
// 3. Decomposition.  When no Clifford rule applies, one remaining T-like spider (odd phase,
//    Section 2.1) becomes a Boolean parameter: z_v is replaced by a new x_k, which makes its
//    neighbours' phases polar in x_k (the plug |x_k> of the cat/stabiliser decomposition), and
//    simplification continues.  T-like spiders that end up isolated are node factors and need
//    no parameter (Lemma 1 is why a T-like phase is never pushed through a polar one).
// 4. Constraints.  A factor 1 + w^{4 (c xor l(x))} is 2 or 0: with constraint elimination on,
//    one parameter of l is solved for and substituted into every form, which halves the term
//    count per constraint without changing the sum.
// 5. Outcome-parametric queries.  With every output bit y_i a parameter, the effect <y_i| is a
//    spider of polar phase pi (c xor y_i) (Section 3.2), the simplification runs unchanged, and
//    the y_i are never solved for: the program's last n parameters are y_0 .. y_{n-1}, so one
//    compilation answers every output string.  A prefix query (the marginal of the first k
//    qubits, the doubled diagram of Fig. 3 right) does the same with the projector
//    |y_i><y_i| on each measured qubit: the effect <y_i| and a fresh spider z_i held equal to
//    y_i by a second polar effect, so the first k outcomes are the program's parameters
//    (the repeated weak simulation of Appendix F).
// The scalar is tracked exactly in Z[w] with a power of sqrt2 throughout.

#include "compiler.h"

#include <algorithm>
#include <cstring>
#include <map>
#include <vector>

namespace {

// ------------------------------------------------------------------ parameter bitsets

constexpr int kParamWords = 4;  // up to 256 parameters while compiling
struct PBits {
    uint64_t w[kParamWords] = {0, 0, 0, 0};
    bool any() const { return w[0] | w[1] | w[2] | w[3]; }
    void flip(int k) { w[k >> 6] ^= (uint64_t)1 << (k & 63); }
    bool test(int k) const { return (w[k >> 6] >> (k & 63)) & 1; }
    PBits &operator^=(const PBits &o) {
        for (int i = 0; i < kParamWords; ++i) w[i] ^= o.w[i];
        return *this;
    }
    bool operator<(const PBits &o) const {
        for (int i = kParamWords - 1; i >= 0; --i)
            if (w[i] != o.w[i]) return w[i] < o.w[i];
        return false;
    }
    bool operator==(const PBits &o) const { return !memcmp(w, o.w, sizeof w); }
    int lowest() const {
        for (int i = 0; i < kParamWords; ++i)
            if (w[i]) return i * 64 + __builtin_ctzll(w[i]);
        return -1;
    }
};

PBits operator^(PBits a, const PBits &b) { return a ^= b; }

int m8(long long v) { return (int)(((v % 8) + 8) % 8); }

struct CompileError {
    int code;
    std::string msg;
};

// ------------------------------------------------------------------ circuit

struct Gate {
    int kind;  // 0 h, 1 phase (k), 2 x, 3 cx, 4 cz
    int k;
    int q0, q1;
};

std::vector<Gate> parse_circuit(const char *text, size_t len, int *n_qubits) {
    std::vector<Gate> gates;
    int n = -1;
    size_t i = 0;
    int line = 0;
    while (i < len) {
        size_t j = i;
        while (j < len && text[j] != '\n') ++j;
        ++line;
        std::string ln(text + i, j - i);
        i = j + 1;
        size_t hash = ln.find('#');
        if (hash != std::string::npos) ln.resize(hash);
        std::vector<std::string> tok;
        size_t s = 0;
        while (s < ln.size()) {
            while (s < ln.size() && isspace((unsigned char)ln[s])) ++s;
            size_t e = s;
            while (e < ln.size() && !isspace((unsigned char)ln[e])) ++e;
            if (e > s) tok.push_back(ln.substr(s, e - s));
            s = e;
        }
        if (tok.empty()) continue;
        auto bad = [&](const std::string &why) {
            return CompileError{SIM_EINVAL, "circuit line " + std::to_string(line) + ": " + why};
        };
        auto qubit = [&](const std::string &t) {
            char *end = nullptr;
            long v = strtol(t.c_str(), &end, 10);
            if (*end || t.empty()) throw bad("bad qubit '" + t + "'");
            if (v < 0 || v >= n) throw bad("qubit " + t + " out of range");
            return (int)v;
        };
        std::string g = tok[0];
        for (auto &ch : g) ch = (char)tolower((unsigned char)ch);
        if (g == "qubits") {
            if (n >= 0) throw bad("'qubits' given twice");
            if (tok.size() != 2) throw bad("expected 'qubits <n>'");
            char *end = nullptr;
            long v = strtol(tok[1].c_str(), &end, 10);
            if (*end || v < 1 || v > 4096) throw bad("bad qubit count");
            n = (int)v;
            continue;
        }
        if (n < 0) throw bad("gate before 'qubits'");
        static const std::map<std::string, int> phase = {{"s", 2}, {"sdg", 6}, {"t", 1}, {"tdg", 7}, {"z", 4}};
        Gate G{0, 0, 0, 0};
        if (g == "h" || g == "x" || phase.count(g)) {
            if (tok.size() != 2) throw bad("expected one qubit");
            G.q0 = qubit(tok[1]);
            if (g == "h") G.kind = 0;
            else if (g == "x") G.kind = 2;
            else {
                G.kind = 1;
                G.k = phase.at(g);
            }
        } else if (g == "cx" || g == "cnot" || g == "cz") {
            if (tok.size() != 3) throw bad("expected two qubits");
            G.kind = g == "cz" ? 4 : 3;
            G.q0 = qubit(tok[1]);
            G.q1 = qubit(tok[2]);
            if (G.q0 == G.q1) throw bad("two-qubit gate on one qubit");
        } else {
            throw bad("unknown gate '" + tok[0] + "'");
        }
        gates.push_back(G);
    }
    if (n < 0) throw CompileError{SIM_EINVAL, "circuit: missing 'qubits <n>'"};
    *n_qubits = n;
    return gates;
}

// ------------------------------------------------------------------ exact scalar

struct Scalar {
    Zw c = zw_one();
    int32_t e = 0;  // value = c * sqrt2^e
    bool zero = false;
    void mul(const Zw &f) {
        if (zero) return;
        Zw r;
        if (!zw_mul_checked(c, f, &r)) throw CompileError{SIM_ERANGE, "scalar exceeds int128"};
        c = r;
        if (zw_is_zero(c)) {
            zero = true;
            return;
        }
        zw_canonicalise(&c, &e);
    }
    void rot(int k) { c = zw_rot(c, m8(k)); }
    void one_plus_w(int k) {  // times 1 + w^k
        k = m8(k);
        if (k == 0) e += 2;
        else if (k == 4) zero = true;
        else if (k == 2) {
            e += 1;
            rot(1);
        } else if (k == 6) {
            e += 1;
            rot(7);
        } else {
            Zw f = zw_rot(zw_one(), k);
            f.c[0] += 1;
            mul(f);
        }
    }
};

// ------------------------------------------------------------------ path-sum builder

struct Label {
    std::vector<int> S;  // sorted spider ids
    int c = 0;
};

std::vector<int> sym_diff(const std::vector<int> &a, const std::vector<int> &b) {
    std::vector<int> r;
    std::set_symmetric_difference(a.begin(), a.end(), b.begin(), b.end(), std::back_inserter(r));
    return r;
}

struct Builder {
    int nv = 0;
    std::vector<int> phase;                      // a_v
    std::vector<std::pair<int, int>> toggles;    // Hadamard edges, toggled
    std::map<std::vector<int>, int> pm;          // phase on a parity of spiders
    std::vector<std::pair<int, int>> polar;      // (spider, parameter): phase + pi x_parameter
    Scalar sc;

    int new_spider(int a) {
        phase.push_back(m8(a));
        return nv++;
    }
    // phase k (units of pi/4) on the affine parity L
    void add_phase(const Label &L, int k) {
        k = m8(k);
        if (!k) return;
        if (L.S.empty()) {
            if (L.c) sc.rot(k);
            return;
        }
        if (L.c) {  // k (1 xor P) = k - k P
            sc.rot(k);
            pm[L.S] = m8(pm[L.S] - k);
        } else {
            pm[L.S] = m8(pm[L.S] + k);
        }
    }
    // H on a wire with parity L: new spider joined to every spider of L, phase pi if c
    Label hadamard(const Label &L) {
        int z = new_spider(L.c ? 4 : 0);
        for (int s : L.S) toggles.push_back({z, s});
        sc.e -= 1;
        return Label{{z}, 0};
    }
    // <y| on a wire with parity L (or a projector): delta(L = y) = 1/2 sum_h (-1)^{h (L xor y)}
    void constrain(const Label &L, int y) {
        if (L.S.empty()) {
            if ((L.c ^ y) & 1) sc.zero = true;
            return;
        }
        int h = new_spider(((L.c ^ y) & 1) ? 4 : 0);
        for (int s : L.S) toggles.push_back({h, s});
        sc.e -= 2;
    }
    // <y| with y = parameter k: the spider of the effect gets the polar phase pi (c xor x_k)
    void constrain_param(const Label &L, int k) {
        int h = new_spider((L.c & 1) ? 4 : 0);
        for (int s : L.S) toggles.push_back({h, s});
        polar.push_back({h, k});
        sc.e -= 2;
    }
    // phases on parities -> graph-like form
    void flush_phases() {
        for (const auto &kv : pm) {
            const std::vector<int> &S = kv.first;
            int k = m8(kv.second);
            if (!k) continue;
            if (S.size() == 1) {
                phase[S[0]] = m8(phase[S[0]] + k);
            } else if (k % 2 == 0) {
                // k * parity = k sum z - 2k sum_{pairs} z z (mod 8) for even k
                for (int s : S) phase[s] = m8(phase[s] + k);
                if (k % 4 == 2)
                    for (size_t i = 0; i < S.size(); ++i)
                        for (size_t j = i + 1; j < S.size(); ++j) toggles.push_back({S[i], S[j]});
            } else {
                // phase gadget: w^{k P} = 1/2 sum_{g,h} w^{k g} (-1)^{h (g xor P)}
                int g = new_spider(k);
                int h = new_spider(0);
                toggles.push_back({h, g});
                for (int s : S) toggles.push_back({h, s});
                sc.e -= 2;
            }
        }
        pm.clear();
    }
};

// ------------------------------------------------------------------ graph and rules

struct Form {
    PBits m;
    int c = 0;
};

struct Emitted {
    std::vector<std::pair<Form, int>> nodes;  // (form, a): factor 1 + w^{a + 4 l(x)}
    std::vector<std::pair<Form, int>> lins;   // (form, c): phase c l(x)
};

struct Graph {
    int n = 0, words = 0;
    std::vector<uint64_t> adj;  // n rows of `words` words
    std::vector<int> a;
    std::vector<PBits> l;
    std::vector<char> alive;
    std::vector<int> deg;
    int n_params = 0;
    int t_like = 0;
    bool hub_params = false;  // a parameter may go to a spider whose T-like leaves it isolates
    Scalar *sc = nullptr;
    Emitted *em = nullptr;

    uint64_t *row(int v) { return adj.data() + (size_t)v * words; }
    bool edge(int u, int v) { return (row(u)[v >> 6] >> (v & 63)) & 1; }
    void toggle(int u, int v) {
        row(u)[v >> 6] ^= (uint64_t)1 << (v & 63);
        row(v)[u >> 6] ^= (uint64_t)1 << (u & 63);
        int d = edge(u, v) ? 1 : -1;
        deg[u] += d;
        deg[v] += d;
    }
    std::vector<int> nbrs(int v) {
        std::vector<int> r;
        const uint64_t *rw = row(v);
        for (int i = 0; i < words; ++i) {
            uint64_t x = rw[i];
            while (x) {
                int b = __builtin_ctzll(x);
                r.push_back(i * 64 + b);
                x &= x - 1;
            }
        }
        return r;
    }
    void remove(int v) {
        for (int u : nbrs(v)) toggle(u, v);
        alive[v] = 0;
    }

    // phase c * form, folded into the scalar when the form is constant
    void lin(const Form &f, int c) {
        c = m8(c);
        if (!c) return;
        if (!f.m.any()) {
            if (f.c) sc->rot(c);
            return;
        }
        em->lins.push_back({f, c});
    }
    // phase 4 * f1 * f2 for two affine forms
    void quad4(const Form &f1, const Form &f2) {
        if (!f1.m.any()) {
            if (f1.c) lin(f2, 4);
            return;
        }
        if (!f2.m.any()) {
            if (f2.c) lin(f1, 4);
            return;
        }
        lin(f1, 2);
        lin(f2, 2);
        lin(Form{f1.m ^ f2.m, f1.c ^ f2.c}, 6);
    }

    bool pauli(int v) { return a[v] % 4 == 0; }
    bool proper_clifford(int v) { return a[v] == 2 || a[v] == 6; }

    void rule_isolated(int v) {
        if (!l[v].any()) sc->one_plus_w(a[v]);
        else if (a[v] == 2 || a[v] == 6) {
            // 1 + w^{2s + 4l} = sqrt2 w^{s} w^{-2 s l}
            int s = a[v] == 2 ? 1 : -1;
            sc->e += 1;
            sc->rot(s);
            lin(Form{l[v], 0}, -2 * s);
        } else {
            em->nodes.push_back({Form{l[v], 0}, a[v]});
        }
        alive[v] = 0;
    }

    void rule_lc(int v) {
        int s = a[v] == 2 ? 1 : -1;
        std::vector<int> N = nbrs(v);
        sc->e += 1;
        sc->rot(s);
        if (l[v].any()) lin(Form{l[v], 0}, -2 * s);
        for (int u : N) {
            a[u] = m8(a[u] - 2 * s);
            l[u] ^= l[v];
        }
        remove(v);
        for (size_t i = 0; i < N.size(); ++i)
            for (size_t j = i + 1; j < N.size(); ++j) toggle(N[i], N[j]);
    }

    void rule_pivot(int u, int v) {
        const int cu = a[u] / 4, cv = a[v] / 4;
        const Form Au{l[u], cu}, Av{l[v], cv};
        std::vector<int> Nu = nbrs(u), Nv = nbrs(v);
        Nu.erase(std::remove(Nu.begin(), Nu.end(), v), Nu.end());
        Nv.erase(std::remove(Nv.begin(), Nv.end(), u), Nv.end());
        sc->e += 2;
        quad4(Au, Av);
        std::vector<char> inU(n, 0), inV(n, 0);
        for (int w : Nu) inU[w] = 1;
        for (int w : Nv) inV[w] = 1;
        for (int w : Nv) {
            a[w] = m8(a[w] + 4 * cu);
            l[w] ^= l[u];
        }
        for (int w : Nu) {
            a[w] = m8(a[w] + 4 * cv);
            l[w] ^= l[v];
            if (inV[w]) a[w] = m8(a[w] + 4);
        }
        remove(u);
        remove(v);
        std::vector<int> A, B, C;
        for (int w : Nu) (inV[w] ? C : A).push_back(w);
        for (int w : Nv)
            if (!inU[w]) B.push_back(w);
        for (int x : A)
            for (int y : B) toggle(x, y);
        for (int x : A)
            for (int y : C) toggle(x, y);
        for (int x : B)
            for (int y : C) toggle(x, y);
    }

    // Pauli u with the single neighbour v: z_v = cu xor l_u(x)
    void rule_leaf(int u, int v) {
        const Form F{l[u], a[u] / 4};
        sc->e += 2;
        lin(F, a[v]);
        quad4(Form{l[v], 0}, F);
        for (int w : nbrs(v)) {
            if (w == u) continue;
            a[w] = m8(a[w] + 4 * F.c);
            l[w] ^= F.m;
        }
        remove(u);
        remove(v);
    }

    // Pauli u with l_u = 0 and neighbours v, w: z_w = z_v xor cu; w merges into v
    void rule_fuse(int u, int v, int w) {
        const int cu = a[u] / 4;
        sc->e += 2;
        remove(u);
        std::vector<int> Nw = nbrs(w);
        if (!cu) {
            a[v] = m8(a[v] + a[w]);
            l[v] ^= l[w];
            for (int t : Nw) {
                if (t == v) a[v] = m8(a[v] + 4);
                else toggle(v, t);
            }
        } else {
            // z_w = 1 - z_v
            sc->rot(a[w]);
            a[v] = m8(a[v] - a[w]);
            if (l[w].any()) lin(Form{l[w], 0}, 4);
            l[v] ^= l[w];
            for (int t : Nw) {
                if (t == v) continue;
                a[t] = m8(a[t] + 4);
                toggle(v, t);
            }
        }
        remove(w);
    }

    void rule_param(int v, int p_limit) {
        if (n_params >= kParamWords * 64 || n_params >= p_limit)
            throw CompileError{SIM_ERANGE, "more than " + std::to_string(std::min(p_limit, kParamWords * 64)) +
                                               " parameters before constraint elimination"};
        int k = n_params++;
        PBits ek;
        ek.flip(k);
        lin(Form{ek, 0}, a[v]);
        quad4(Form{l[v], 0}, Form{ek, 0});
        for (int u : nbrs(v)) l[u] ^= ek;
        remove(v);
    }

    bool step(int p_limit) {
        // isolated spiders, then local complementation, pivots, leaves, fusions
        for (int v = 0; v < n; ++v)
            if (alive[v] && deg[v] == 0) {
                rule_isolated(v);
                return true;
            }
        for (int v = 0; v < n; ++v)
            if (alive[v] && proper_clifford(v)) {
                rule_lc(v);
                return true;
            }
        for (int u = 0; u < n; ++u) {
            if (!alive[u] || !pauli(u)) continue;
            for (int v : nbrs(u))
                if (pauli(v)) {
                    rule_pivot(u, v);
                    return true;
                }
        }
        for (int u = 0; u < n; ++u)
            if (alive[u] && pauli(u) && deg[u] == 1) {
                rule_leaf(u, nbrs(u)[0]);
                return true;
            }
        for (int u = 0; u < n; ++u)
            if (alive[u] && pauli(u) && deg[u] == 2 && !l[u].any()) {
                std::vector<int> N = nbrs(u);
                rule_fuse(u, N[0], N[1]);
                return true;
            }
        // decomposition: parameterise one spider.  Its T-like neighbours of degree 1 are then
        // isolated, i.e. node factors needing no parameter of their own, so the spider that
        // removes the most T-like spiders (itself if T-like, plus those neighbours) is taken;
        // ties go to a T-like spider, then to the highest degree
        int best = -1, best_gain = 0;
        for (int v = 0; v < n; ++v) {
            if (!alive[v]) continue;
            int gain = a[v] & 1;
            if (hub_params)
                for (int u : nbrs(v)) gain += (a[u] & 1) && deg[u] == 1;
            if (!gain) continue;
            const bool better = best < 0 || gain > best_gain ||
                                (gain == best_gain && ((a[v] & 1) > (a[best] & 1) ||
                                                       ((a[v] & 1) == (a[best] & 1) && deg[v] > deg[best])));
            if (better) {
                best = v;
                best_gain = gain;
            }
        }
        if (best >= 0) {
            rule_param(best, p_limit);
            return true;
        }
        return false;
    }
};

// ------------------------------------------------------------------ IR emission

// Parameters 0 .. n_outer-1 are query parameters: never eliminated, emitted last (in order).
void emit_ir(const Emitted &em, int n_params, int n_outer, const Scalar &sc, bool eliminate, int p_cap,
             IrProgram *out, CompileStats *stats) {
    Scalar s = sc;
    std::vector<std::pair<Form, int>> nodes = em.nodes, lins = em.lins;
    std::vector<char> gone(n_params, 0);
    int n_constraints = 0;
    if (eliminate) {
        std::vector<std::pair<Form, int>> kept;
        for (size_t i = 0; i < nodes.size(); ++i) {
            Form f = nodes[i].first;
            int a = nodes[i].second;
            if (a % 4 != 0) {
                kept.push_back(nodes[i]);
                continue;
            }
            if (!f.m.any()) {
                s.one_plus_w(a + 4 * f.c);
                continue;
            }
            // nonzero iff l(x) = a/4: solve for the lowest decomposition parameter of l (a
            // constraint on query parameters alone stays a factor)
            int k = -1;
            for (int b = n_outer; b < n_params && k < 0; ++b)
                if (f.m.test(b)) k = b;
            if (k < 0) {
                kept.push_back(nodes[i]);
                continue;
            }
            const int rhs = (a / 4) ^ f.c;
            auto subst = [&](Form &g) {
                if (g.m.test(k)) {
                    g.m ^= f.m;
                    g.c ^= rhs;
                }
            };
            for (size_t j = i + 1; j < nodes.size(); ++j) subst(nodes[j].first);
            for (auto &kn : kept) subst(kn.first);
            for (auto &ln : lins) subst(ln.first);
            s.e += 2;
            gone[k] = 1;
            ++n_constraints;
        }
        nodes = kept;
    }
    // renumber surviving parameters: decomposition parameters first, then the query parameters
    std::vector<int> newidx(n_params, -1);
    int p = 0;
    for (int k = n_outer; k < n_params; ++k)
        if (!gone[k]) newidx[k] = p++;
    const int p_decomp = p;
    for (int k = 0; k < n_outer; ++k) newidx[k] = p++;
    if (p > 62) throw CompileError{SIM_ERANGE, "p = " + std::to_string(p) + " exceeds 62"};
    if (p_decomp > p_cap)
        throw CompileError{SIM_ERANGE, "p = " + std::to_string(p_decomp) + " exceeds the cap " + std::to_string(p_cap)};
    auto remap = [&](const PBits &m) {
        uint64_t r = 0;
        for (int k = 0; k < n_params; ++k)
            if (m.test(k)) r |= (uint64_t)1 << newidx[k];
        return r;
    };
    IrProgram P;
    P.p = p;
    P.outer = n_outer;
    std::map<std::pair<uint64_t, int>, int> form_ids;
    auto form_of = [&](const Form &f) {
        auto key = std::make_pair(remap(f.m), f.c);
        auto it = form_ids.find(key);
        if (it != form_ids.end()) return it->second;
        int id = (int)P.forms.size();
        P.forms.push_back(IrForm{f.c, key.first});
        form_ids[key] = id;
        return id;
    };
    std::map<int, int> lin_acc;
    for (const auto &ln : lins) {
        if (!ln.first.m.any()) {
            if (ln.first.c) s.rot(ln.second);
            continue;
        }
        int id = form_of(ln.first);
        lin_acc[id] = m8(lin_acc[id] + ln.second);
    }
    for (const auto &nd : nodes) {
        if (!nd.first.m.any()) {
            s.one_plus_w(nd.second + 4 * nd.first.c);
            continue;
        }
        P.nodes.push_back(IrNode{form_of(nd.first), nd.second, 4});
    }
    for (const auto &kv : lin_acc)
        if (kv.second) P.lin.push_back(IrLin{kv.second, kv.first});
    if (s.zero) {
        P.forms.clear();
        P.nodes.clear();
        P.lin.clear();
        P.scalar = zw_zero();
        P.e = 0;
    } else {
        P.scalar = s.c;
        P.e = s.e;
    }
    stats->n_constraints = n_constraints;
    stats->n_params = p;
    *out = std::move(P);
}

}  // namespace

int compile_circuit(const char *text, size_t len, const sim_query &q, const CompileOptions &opts, IrProgram *out,
                    CompileStats *stats, std::string *err) {
    try {
        int n = 0;
        std::vector<Gate> gates = parse_circuit(text, len, &n);
        if (q.n_qubits != (uint32_t)n)
            throw CompileError{SIM_EINVAL, "query has " + std::to_string(q.n_qubits) + " qubits, circuit has " +
                                               std::to_string(n)};
        std::vector<Gate> seq;
        // doubled diagrams: the measured qubits, each with a fixed value (0/1) or, as a
        // projector |y_i><y_i| with y_i a query parameter, -1
        std::vector<std::pair<int, int>> proj;
        size_t proj_at = 0;
        int n_outer = 0;
        if (q.kind == SIM_QUERY_AMPLITUDE) {
            if (!q.out_bits) throw CompileError{SIM_EINVAL, "amplitude query without output bits"};
            for (int i = 0; i < n; ++i)
                if (q.out_bits[i] > 1) throw CompileError{SIM_EINVAL, "output bits must be 0 or 1"};
            seq = gates;
        } else if (q.kind == SIM_QUERY_OUTCOMES) {
            if (n > 62) throw CompileError{SIM_ERANGE, "more than 62 output parameters"};
            n_outer = n;
            seq = gates;
        } else if (q.kind == SIM_QUERY_MARGINAL || q.kind == SIM_QUERY_PREFIX) {
            if (q.kind == SIM_QUERY_MARGINAL) {
                if (q.qubit >= (uint32_t)n || q.value > 1) throw CompileError{SIM_EINVAL, "bad marginal query"};
                proj.push_back({(int)q.qubit, (int)q.value});
            } else {
                const int k = (int)q.qubit;
                if (k < 1 || k > n) throw CompileError{SIM_EINVAL, "prefix length must be 1 .. n_qubits"};
                if (!q.out_bits && k > 62) throw CompileError{SIM_ERANGE, "more than 62 prefix parameters"};
                for (int i = 0; i < k; ++i) {
                    if (q.out_bits && q.out_bits[i] > 1) throw CompileError{SIM_EINVAL, "prefix bits must be 0 or 1"};
                    proj.push_back({i, q.out_bits ? (int)q.out_bits[i] : -1});
                }
                if (!q.out_bits) n_outer = k;
            }
            // <0| C^dag P C |0>: gates outside the backward light cone of the measured qubits
            // cancel against their adjoints, so only the light cone is doubled
            std::vector<char> rel(n, 0);
            for (const auto &pq : proj) rel[pq.first] = 1;
            std::vector<Gate> cone;
            for (size_t i = gates.size(); i-- > 0;) {
                const Gate &G = gates[i];
                bool two = G.kind >= 3;
                if (rel[G.q0] || (two && rel[G.q1])) {
                    cone.push_back(G);
                    if (two) rel[G.q0] = rel[G.q1] = 1;
                }
            }
            std::reverse(cone.begin(), cone.end());
            seq = cone;
            proj_at = seq.size();
            for (size_t i = cone.size(); i-- > 0;) {
                Gate G = cone[i];
                if (G.kind == 1) G.k = m8(-G.k);
                seq.push_back(G);
            }
        } else {
            throw CompileError{SIM_EINVAL, "unknown query kind"};
        }

        Builder B;
        std::vector<Label> wire(n);
        for (size_t i = 0; i <= seq.size(); ++i) {
            if (!proj.empty() && i == proj_at) {
                for (const auto &pq : proj) {
                    const int w = pq.first;
                    if (pq.second >= 0) {
                        B.constrain(wire[w], pq.second);
                        wire[w] = Label{{}, pq.second};
                    } else {
                        // |y><y| with y = parameter w: the effect <y|, then |y> as a fresh
                        // spider z held equal to y by a second polar effect
                        B.constrain_param(wire[w], w);
                        const int z = B.new_spider(0);
                        wire[w] = Label{{z}, 0};
                        B.constrain_param(wire[w], w);
                    }
                }
            }
            if (i == seq.size()) break;
            const Gate &G = seq[i];
            switch (G.kind) {
                case 0: wire[G.q0] = B.hadamard(wire[G.q0]); break;
                case 1: B.add_phase(wire[G.q0], G.k); break;
                case 2: wire[G.q0].c ^= 1; break;
                case 3:
                    wire[G.q1].S = sym_diff(wire[G.q1].S, wire[G.q0].S);
                    wire[G.q1].c ^= wire[G.q0].c;
                    break;
                case 4: {
                    // 4 A B = 2 A + 2 B - 2 (A xor B)
                    const Label &A = wire[G.q0], &Bq = wire[G.q1];
                    Label X{sym_diff(A.S, Bq.S), A.c ^ Bq.c};
                    B.add_phase(A, 2);
                    B.add_phase(Bq, 2);
                    B.add_phase(X, 6);
                    break;
                }
            }
        }
        for (int i = 0; i < n; ++i) {
            if (q.kind == SIM_QUERY_OUTCOMES) B.constrain_param(wire[i], i);
            else B.constrain(wire[i], q.kind == SIM_QUERY_AMPLITUDE ? (int)q.out_bits[i] : 0);
        }
        B.flush_phases();

        Emitted em;
        Scalar sc = B.sc;
        int t_like = 0;
        int n_params = 0;
        if (!sc.zero) {
            Graph G;
            G.n = B.nv;
            G.words = (G.n + 63) / 64 + 1;
            G.adj.assign((size_t)G.n * G.words, 0);
            G.a = B.phase;
            G.l.assign(G.n, PBits());
            G.alive.assign(G.n, 1);
            G.deg.assign(G.n, 0);
            G.sc = &sc;
            G.em = &em;
            for (const auto &t : B.toggles) G.toggle(t.first, t.second);
            for (const auto &pv : B.polar) G.l[pv.first].flip(pv.second);
            G.n_params = n_outer;  // parameters 0 .. n_outer-1 are the output bits
            G.hub_params = opts.hub_params;
            for (int v = 0; v < G.n; ++v) t_like += G.a[v] & 1;
            const int p_limit = kParamWords * 64;
            while (!sc.zero && G.step(p_limit)) {
            }
            n_params = G.n_params;
        }
        stats->t_count = t_like;
        emit_ir(em, std::max(n_params, n_outer), n_outer, sc, opts.eliminate_constraints, opts.p_cap, out, stats);
    } catch (const CompileError &ce) {
        *err = ce.msg;
        return ce.code;
    }
    return SIM_OK;
}
