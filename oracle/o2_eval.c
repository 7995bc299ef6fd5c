/*
 * Term-by-term CPU evaluator of a parametric scalar: TEST INFRASTRUCTURE ONLY.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg run this program.
 * It shares no code with the GPU library and is deliberately plain and slow.
 *
 * What it computes (the parametric scalar expression of the paper's Eq. 2, with every
 * decomposition term indexed by a Boolean assignment x of the p parameters):
 *
 *     S = c * sum_{x in {0,1}^p} w^{phi(x)} * prod_j F_j(x),     w = e^{i pi/4}
 *
 *   - a form is l(x) = const XOR parity(mask AND x)  (the polar phase of Eq. 1: the phase
 *     is alpha + pi * l(x));
 *   - a node factor is 1 + w^{a + b l(x)} (the "node" subterm of the Appendix C table,
 *     with b = 4 giving 1 + e^{i(alpha + pi l)});
 *   - a pair factor is 1 + w^{a+4 l1} + w^{b+4 l2} - w^{a+b+4(l1 XOR l2)} (the phase-pair
 *     subterm of Eq. 3 with Psi = a pi/4 + pi l1 and Phi = b pi/4 + pi l2);
 *   - phi(x) = sum of c * l_f(x) over linear terms plus c * x_i x_j ... over variable
 *     monomials, taken mod 8 (the pi-pair and half-pi subterms of the same table are such
 *     phase terms);
 *   - c = c0 + c1 w + c2 w^2 + c3 w^3.
 *
 * Numbers are exact elements of Z[w] held as four __int128 coefficients in the basis
 * 1, w, w^2, w^3 (w^4 = -1).  Each factor value is built from its definition and
 * multiplied in with the full product of Z[w] (no rotation shortcut, no value classes);
 * terms are visited in plain binary order x = first .. first+count-1 and summed.  Any
 * int128 overflow aborts the run (exit status 3) instead of wrapping.
 *
 * Input: the "zxir 1" text on stdin.  Output lines:
 *     raw <r0> <r1> <r2> <r3>            the sum without c and sqrt2^e
 *     value <v0> <v1> <v2> <v3> <e>      c times the sum, times sqrt2^e
 *     term <x> <t0> <t1> <t2> <t3>       one line per assignment with --terms
 * Options: --threads T, --first F --count N (assignment range), --perm i0,i1,...
 * (bit j of the assignment index sets variable perm[j]; default identity), --terms,
 * --points x0,c0,c1,..,c_{k-1} (hex; instead of --perm: index t names the assignment
 * x0 XOR the c_j of the set bits j of t, 0 <= t < 2^k, so a range of indices is a set of
 * points of an affine subspace; the terms are evaluated exactly as for any other index).
 */
#include <ctype.h>
#include <pthread.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef __int128 i128;

typedef struct {
    i128 c[4];
} zw;

static void die(const char *msg) {
    fprintf(stderr, "o2_eval: %s\n", msg);
    exit(2);
}

static void overflow(void) {
    fprintf(stderr, "o2_eval: int128 overflow\n");
    exit(3);
}

static i128 add_chk(i128 a, i128 b) {
    i128 r;
    if (__builtin_add_overflow(a, b, &r)) overflow();
    return r;
}

static i128 mul_chk(i128 a, i128 b) {
    i128 r;
    if (__builtin_mul_overflow(a, b, &r)) overflow();
    return r;
}

static zw zw_zero(void) {
    zw z;
    memset(&z, 0, sizeof z);
    return z;
}

/* w^k as an element of Z[w]: w^k for k < 4, and -w^(k-4) for 4 <= k < 8 */
static zw zw_omega_pow(int k) {
    zw z = zw_zero();
    k = ((k % 8) + 8) % 8;
    if (k < 4)
        z.c[k] = 1;
    else
        z.c[k - 4] = -1;
    return z;
}

static zw zw_add(zw a, zw b) {
    zw r;
    for (int i = 0; i < 4; i++) r.c[i] = add_chk(a.c[i], b.c[i]);
    return r;
}

static zw zw_sub(zw a, zw b) {
    zw r;
    for (int i = 0; i < 4; i++) {
        i128 nb;
        if (__builtin_sub_overflow((i128)0, b.c[i], &nb)) overflow();
        r.c[i] = add_chk(a.c[i], nb);
    }
    return r;
}

/* product in Z[w] = Z[X]/(X^4 + 1): w^i * w^j = w^(i+j), and w^(i+j) = -w^(i+j-4) */
static zw zw_mul(zw a, zw b) {
    zw r = zw_zero();
    for (int i = 0; i < 4; i++) {
        for (int j = 0; j < 4; j++) {
            i128 t = mul_chk(a.c[i], b.c[j]);
            if (i + j < 4) {
                r.c[i + j] = add_chk(r.c[i + j], t);
            } else {
                i128 nt;
                if (__builtin_sub_overflow((i128)0, t, &nt)) overflow();
                r.c[i + j - 4] = add_chk(r.c[i + j - 4], nt);
            }
        }
    }
    return r;
}

/* ---------------------------------------------------------------- program */

typedef struct {
    int constant;
    uint64_t mask;
} form_t;

typedef struct {
    int form, a, b;
} node_t;

typedef struct {
    int f1, f2, a, b;
} pair_t;

typedef struct {
    int c, form;
} lin_t;

typedef struct {
    int c, deg;
    int vars[8];
} mono_t;

typedef struct {
    int p;
    int n_forms, n_nodes, n_pairs, n_lin, n_mono;
    form_t *forms;
    node_t *nodes;
    pair_t *pairs;
    lin_t *lin;
    mono_t *mono;
    zw scalar;
    int sqrt2_exp;
} program_t;

/* tokenizer over the input text; comments ('#' to end of line) are blanked first */
typedef struct {
    char *buf;
    size_t pos, len;
} lexer_t;

static void blank_comments(char *buf, size_t len) {
    for (size_t i = 0; i < len; i++) {
        if (buf[i] == '#') {
            while (i < len && buf[i] != '\n') buf[i++] = ' ';
        }
    }
}

static char *next_tok(lexer_t *lx) {
    while (lx->pos < lx->len && isspace((unsigned char)lx->buf[lx->pos])) lx->pos++;
    if (lx->pos >= lx->len) return NULL;
    char *start = lx->buf + lx->pos;
    while (lx->pos < lx->len && !isspace((unsigned char)lx->buf[lx->pos])) lx->pos++;
    if (lx->pos < lx->len) lx->buf[lx->pos++] = '\0';
    return start;
}

static char *expect_tok(lexer_t *lx) {
    char *t = next_tok(lx);
    if (!t) die("unexpected end of input");
    return t;
}

static void expect_word(lexer_t *lx, const char *w) {
    char *t = expect_tok(lx);
    if (strcmp(t, w) != 0) {
        fprintf(stderr, "o2_eval: expected '%s', got '%s'\n", w, t);
        exit(2);
    }
}

static long long parse_int(lexer_t *lx) {
    char *t = expect_tok(lx);
    char *end;
    long long v = strtoll(t, &end, 10);
    if (*end) die("bad integer");
    return v;
}

static i128 parse_i128(lexer_t *lx) {
    char *t = expect_tok(lx);
    int neg = 0;
    if (*t == '-') {
        neg = 1;
        t++;
    }
    if (!*t) die("bad integer");
    i128 v = 0;
    for (; *t; t++) {
        if (!isdigit((unsigned char)*t)) die("bad integer");
        v = add_chk(mul_chk(v, 10), *t - '0');
    }
    return neg ? -v : v;
}

static uint64_t parse_hex(lexer_t *lx) {
    char *t = expect_tok(lx);
    char *end;
    unsigned long long v = strtoull(t, &end, 16);
    if (*end) die("bad hex mask");
    return (uint64_t)v;
}

static void check_form(const program_t *P, int f) {
    if (f < 0 || f >= P->n_forms) die("form index out of range");
}

static void read_program(program_t *P) {
    size_t cap = 1 << 16, len = 0;
    char *buf = malloc(cap);
    size_t got;
    while ((got = fread(buf + len, 1, cap - len - 1, stdin)) > 0) {
        len += got;
        if (len + 1 >= cap) {
            cap *= 2;
            buf = realloc(buf, cap);
        }
    }
    buf[len] = '\0';
    blank_comments(buf, len);
    lexer_t lx = {buf, 0, len};

    expect_word(&lx, "zxir");
    if (parse_int(&lx) != 1) die("unsupported version");
    expect_word(&lx, "p");
    P->p = (int)parse_int(&lx);
    if (P->p < 0 || P->p > 62) die("p out of range");

    /* optional: the last K parameters are query parameters; a query fixes them, which is a
       range of the binary order here, so the sum itself is unchanged */
    char *t = expect_tok(&lx);
    if (strcmp(t, "outer") == 0) {
        long long k = parse_int(&lx);
        if (k < 0 || k > P->p) die("outer out of range");
        t = expect_tok(&lx);
    }
    if (strcmp(t, "forms") != 0) {
        fprintf(stderr, "o2_eval: expected 'forms', got '%s'\n", t);
        exit(2);
    }
    P->n_forms = (int)parse_int(&lx);
    P->forms = calloc(P->n_forms + 1, sizeof(form_t));
    for (int i = 0; i < P->n_forms; i++) {
        expect_word(&lx, "f");
        P->forms[i].constant = (int)parse_int(&lx) & 1;
        P->forms[i].mask = parse_hex(&lx);
        if (P->p < 64 && (P->forms[i].mask >> P->p)) die("form mask names a variable >= p");
    }
    expect_word(&lx, "nodes");
    P->n_nodes = (int)parse_int(&lx);
    P->nodes = calloc(P->n_nodes + 1, sizeof(node_t));
    for (int i = 0; i < P->n_nodes; i++) {
        expect_word(&lx, "n");
        P->nodes[i].form = (int)parse_int(&lx);
        P->nodes[i].a = (int)parse_int(&lx);
        P->nodes[i].b = (int)parse_int(&lx);
        check_form(P, P->nodes[i].form);
    }
    expect_word(&lx, "pairs");
    P->n_pairs = (int)parse_int(&lx);
    P->pairs = calloc(P->n_pairs + 1, sizeof(pair_t));
    for (int i = 0; i < P->n_pairs; i++) {
        expect_word(&lx, "q");
        P->pairs[i].f1 = (int)parse_int(&lx);
        P->pairs[i].f2 = (int)parse_int(&lx);
        P->pairs[i].a = (int)parse_int(&lx);
        P->pairs[i].b = (int)parse_int(&lx);
        check_form(P, P->pairs[i].f1);
        check_form(P, P->pairs[i].f2);
    }
    expect_word(&lx, "lin");
    P->n_lin = (int)parse_int(&lx);
    P->lin = calloc(P->n_lin + 1, sizeof(lin_t));
    for (int i = 0; i < P->n_lin; i++) {
        expect_word(&lx, "l");
        P->lin[i].c = (int)parse_int(&lx);
        P->lin[i].form = (int)parse_int(&lx);
        check_form(P, P->lin[i].form);
    }
    expect_word(&lx, "mono");
    P->n_mono = (int)parse_int(&lx);
    P->mono = calloc(P->n_mono + 1, sizeof(mono_t));
    for (int i = 0; i < P->n_mono; i++) {
        expect_word(&lx, "m");
        P->mono[i].c = (int)parse_int(&lx);
        P->mono[i].deg = (int)parse_int(&lx);
        if (P->mono[i].deg < 0 || P->mono[i].deg > 8) die("monomial degree out of range");
        for (int k = 0; k < P->mono[i].deg; k++) {
            P->mono[i].vars[k] = (int)parse_int(&lx);
            if (P->mono[i].vars[k] < 0 || P->mono[i].vars[k] >= P->p) die("monomial variable out of range");
        }
    }
    expect_word(&lx, "scalar");
    for (int k = 0; k < 4; k++) P->scalar.c[k] = parse_i128(&lx);
    P->sqrt2_exp = (int)parse_int(&lx);
    expect_word(&lx, "end");
    free(buf);
}

/* ---------------------------------------------------------------- evaluation */

static int form_value(const form_t *f, uint64_t x) {
    return (f->constant ^ __builtin_popcountll(f->mask & x)) & 1;
}

static int var_value(uint64_t x, int v) { return (int)((x >> v) & 1); }

/* one term: the full product of its factors times w^phi, each factor from its definition */
static zw eval_term(const program_t *P, uint64_t x) {
    zw t = zw_omega_pow(0);
    for (int j = 0; j < P->n_nodes; j++) {
        const node_t *n = &P->nodes[j];
        int l = form_value(&P->forms[n->form], x);
        zw f = zw_omega_pow(n->a + n->b * l);
        f.c[0] = add_chk(f.c[0], 1);
        t = zw_mul(t, f);
    }
    for (int j = 0; j < P->n_pairs; j++) {
        const pair_t *q = &P->pairs[j];
        int l1 = form_value(&P->forms[q->f1], x);
        int l2 = form_value(&P->forms[q->f2], x);
        zw f = zw_omega_pow(0);
        f = zw_add(f, zw_omega_pow(q->a + 4 * l1));
        f = zw_add(f, zw_omega_pow(q->b + 4 * l2));
        f = zw_sub(f, zw_omega_pow(q->a + q->b + 4 * (l1 ^ l2)));
        t = zw_mul(t, f);
    }
    long long phi = 0;
    for (int j = 0; j < P->n_lin; j++) phi += (long long)P->lin[j].c * form_value(&P->forms[P->lin[j].form], x);
    for (int j = 0; j < P->n_mono; j++) {
        int prod = 1;
        for (int k = 0; k < P->mono[j].deg; k++) prod &= var_value(x, P->mono[j].vars[k]);
        phi += (long long)P->mono[j].c * prod;
    }
    return zw_mul(t, zw_omega_pow((int)(((phi % 8) + 8) % 8)));
}

typedef struct {
    const program_t *P;
    const int *perm;
    const uint64_t *points;  /* x0, then k columns (--points) */
    int n_points;
    uint64_t first, count;
    int print_terms;
    zw sum;
} job_t;

static uint64_t index_to_assignment(const program_t *P, const int *perm, uint64_t idx) {
    if (!perm) return idx;
    uint64_t x = 0;
    for (int j = 0; j < P->p; j++)
        if ((idx >> j) & 1) x |= (uint64_t)1 << perm[j];
    return x;
}

static void print_i128(FILE *f, i128 v) {
    char tmp[64];
    int n = 0, neg = v < 0;
    unsigned __int128 u = neg ? (unsigned __int128)(-(v + 1)) + 1 : (unsigned __int128)v;
    do {
        tmp[n++] = (char)('0' + (int)(u % 10));
        u /= 10;
    } while (u);
    if (neg) fputc('-', f);
    while (n) fputc(tmp[--n], f);
}

static void *run_job(void *arg) {
    job_t *J = (job_t *)arg;
    zw sum = zw_zero();
    for (uint64_t i = 0; i < J->count; i++) {
        uint64_t idx = J->first + i;
        uint64_t x;
        if (J->points) {
            x = J->points[0];
            for (int j = 0; j < J->n_points; j++)
                if ((idx >> j) & 1) x ^= J->points[1 + j];
        } else {
            x = index_to_assignment(J->P, J->perm, idx);
        }
        zw t = eval_term(J->P, x);
        if (J->print_terms) {
            printf("term %llu", (unsigned long long)idx);
            for (int k = 0; k < 4; k++) {
                putchar(' ');
                print_i128(stdout, t.c[k]);
            }
            putchar('\n');
        }
        sum = zw_add(sum, t);
    }
    J->sum = sum;
    return NULL;
}

int main(int argc, char **argv) {
    int threads = 1, print_terms = 0, have_range = 0;
    unsigned long long first = 0, count = 0;
    const char *perm_arg = NULL, *points_arg = NULL;
    for (int i = 1; i < argc; i++) {
        if (!strcmp(argv[i], "--threads") && i + 1 < argc) threads = atoi(argv[++i]);
        else if (!strcmp(argv[i], "--first") && i + 1 < argc) { first = strtoull(argv[++i], NULL, 10); have_range = 1; }
        else if (!strcmp(argv[i], "--count") && i + 1 < argc) { count = strtoull(argv[++i], NULL, 10); have_range = 1; }
        else if (!strcmp(argv[i], "--perm") && i + 1 < argc) perm_arg = argv[++i];
        else if (!strcmp(argv[i], "--points") && i + 1 < argc) points_arg = argv[++i];
        else if (!strcmp(argv[i], "--terms")) print_terms = 1;
        else die("unknown option");
    }
    program_t P;
    memset(&P, 0, sizeof P);
    read_program(&P);

    uint64_t *points = NULL;
    int n_points = 0;
    if (points_arg) {
        if (perm_arg) die("--points and --perm exclude each other");
        points = calloc(64, sizeof(uint64_t));
        const char *s = points_arg;
        for (int j = 0; j < 64 && *s; j++) {
            char *end;
            unsigned long long v = strtoull(s, &end, 16);
            if (end == s) die("bad --points");
            if (P.p < 64 && (v >> P.p)) die("--points: an assignment outside the p parameters");
            points[j] = v;
            n_points = j;  /* columns after x0 */
            s = end;
            if (*s == ',') s++;
            else if (*s) die("bad --points");
        }
        if (n_points > 62) die("--points: at most 62 columns");
    }
    uint64_t total = (uint64_t)1 << (points ? n_points : P.p);
    if (!have_range) {
        first = 0;
        count = total;
    }
    if (first > total || count > total - first) die("range outside 0 .. 2^p");

    int *perm = NULL;
    if (perm_arg) {
        perm = calloc(P.p + 1, sizeof(int));
        int seen[64] = {0};
        const char *s = perm_arg;
        for (int j = 0; j < P.p; j++) {
            char *end;
            long v = strtol(s, &end, 10);
            if (end == s || v < 0 || v >= P.p || seen[v]) die("bad --perm");
            seen[v] = 1;
            perm[j] = (int)v;
            s = end;
            if (*s == ',') s++;
        }
    }
    if (threads < 1) threads = 1;
    if (print_terms) threads = 1;
    if ((uint64_t)threads > count) threads = count ? (int)count : 1;

    job_t *jobs = calloc(threads, sizeof(job_t));
    pthread_t *tids = calloc(threads, sizeof(pthread_t));
    uint64_t per = count / threads, extra = count % threads, at = first;
    for (int t = 0; t < threads; t++) {
        jobs[t].P = &P;
        jobs[t].perm = perm;
        jobs[t].points = points;
        jobs[t].n_points = n_points;
        jobs[t].first = at;
        jobs[t].count = per + ((uint64_t)t < extra ? 1 : 0);
        jobs[t].print_terms = print_terms;
        at += jobs[t].count;
        pthread_create(&tids[t], NULL, run_job, &jobs[t]);
    }
    zw sum = zw_zero();
    for (int t = 0; t < threads; t++) {
        pthread_join(tids[t], NULL);
        sum = zw_add(sum, jobs[t].sum);
    }
    zw value = zw_mul(P.scalar, sum);
    printf("raw");
    for (int k = 0; k < 4; k++) {
        putchar(' ');
        print_i128(stdout, sum.c[k]);
    }
    printf("\nvalue");
    for (int k = 0; k < 4; k++) {
        putchar(' ');
        print_i128(stdout, value.c[k]);
    }
    printf(" %d\n", P.sqrt2_exp);
    return 0;
}
