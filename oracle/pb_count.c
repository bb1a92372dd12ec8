/* Record counts of the Pauli-boson graph (oracle, plain C).
 *
 * TEST INFRASTRUCTURE ONLY: the oracle's Python code builds the records of
 * small registries; this file only counts, for registries too large for it
 * (the five-mode degree-four graph of Sec. 3.2).  Shares nothing with the GPU
 * library.
 *
 * Labels B_{tau,c,a} = sigma_tau prod_m (b_m^+)^{c_m} b_m^{a_m} (Eq. monomial)
 * are packed as tau + 4 * (c_1 + 64 a_1 + 64^2 c_2 + ...), 6 bits per exponent.
 * The registry holds every label with |c| + |a| <= p (Eq. basis-size).  A
 * commutator [A, B] = AB - BA is expanded term by term: sigma_t sigma_u =
 * i^e sigma_w, and per mode (b^+)^c1 b^a1 (b^+)^c2 b^a2 = sum_k k! C(a1,k) C(c2,k)
 * (b^+)^(c1+c2-k) b^(a1+a2-k); equal labels are merged and zero sums dropped.
 *
 *   E_eta: [B_i, B_j] for i diagonal (tau in {I, z}, c = a), j not: its terms
 *          and the set of labels they reach (the generator registry);
 *   E_L / E_C: [B_a, B_j] for a in the generator registry, j in the registry,
 *          terms inside / outside the registry.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    uint64_t lab;
    int64_t re, im;
} term_t;

static int g_M;

static int expo(uint64_t lab, int m, int which) { /* which 0 = c, 1 = a */
    return (int)((lab >> (2 + 12 * m + 6 * which)) & 63);
}
static uint64_t make_label(int tau, const int* c, const int* a, int M) {
    uint64_t v = (uint64_t)tau;
    for (int m = 0; m < M; ++m) {
        v |= (uint64_t)c[m] << (2 + 12 * m);
        v |= (uint64_t)a[m] << (2 + 12 * m + 6);
    }
    return v;
}
static int64_t fact(int n) { int64_t r = 1; for (int i = 2; i <= n; ++i) r *= i; return r; }
static int64_t choose(int n, int k) {
    if (k < 0 || k > n) return 0;
    int64_t r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}
/* sigma_t sigma_u = i^e sigma_w */
static void pauli(int t, int u, int* w, int* e) {
    if (t == 0) { *w = u; *e = 0; return; }
    if (u == 0) { *w = t; *e = 0; return; }
    if (t == u) { *w = 0; *e = 0; return; }
    *w = 6 - t - u;
    *e = ((t == 1 && u == 2) || (t == 2 && u == 3) || (t == 3 && u == 1)) ? 1 : 3;
}

/* appends sign * (X Y) to buf (unmerged) */
static int product(uint64_t X, uint64_t Y, int sign, term_t* buf, int n, int cap) {
    int M = g_M, w, e;
    pauli((int)(X & 3), (int)(Y & 3), &w, &e);
    static const int pr[4] = {1, 0, -1, 0}, pi[4] = {0, 1, 0, -1};
    /* iterate over the contraction counts k_m by a mixed-radix counter */
    int kmax[8], k[8], c[8], a[8];
    for (int m = 0; m < M; ++m) {
        int a1 = expo(X, m, 1), c2 = expo(Y, m, 0);
        kmax[m] = a1 < c2 ? a1 : c2;
        k[m] = 0;
    }
    for (;;) {
        int64_t f = 1;
        for (int m = 0; m < M; ++m) {
            int c1 = expo(X, m, 0), a1 = expo(X, m, 1), c2 = expo(Y, m, 0), a2 = expo(Y, m, 1);
            f *= fact(k[m]) * choose(a1, k[m]) * choose(c2, k[m]);
            c[m] = c1 + c2 - k[m];
            a[m] = a1 + a2 - k[m];
        }
        if (n >= cap) return -1;
        buf[n].lab = make_label(w, c, a, M);
        buf[n].re = sign * pr[e] * f;
        buf[n].im = sign * pi[e] * f;
        ++n;
        int m = 0;
        while (m < M && k[m] == kmax[m]) k[m++] = 0;
        if (m == M) break;
        ++k[m];
    }
    return n;
}

static int cmp_term(const void* x, const void* y) {
    uint64_t a = ((const term_t*)x)->lab, b = ((const term_t*)y)->lab;
    return a < b ? -1 : a > b;
}
static int cmp_u64(const void* x, const void* y) {
    uint64_t a = *(const uint64_t*)x, b = *(const uint64_t*)y;
    return a < b ? -1 : a > b;
}

/* merged nonzero terms of [A, B] into buf; returns their number (-1: overflow) */
static int commutator(uint64_t A, uint64_t B, term_t* buf, int cap) {
    int n = product(A, B, 1, buf, 0, cap);
    if (n < 0) return -1;
    n = product(B, A, -1, buf, n, cap);
    if (n < 0) return -1;
    qsort(buf, (size_t)n, sizeof(term_t), cmp_term);
    int w = 0;
    for (int r = 0; r < n;) {
        int s = r;
        int64_t re = 0, im = 0;
        while (s < n && buf[s].lab == buf[r].lab) { re += buf[s].re; im += buf[s].im; ++s; }
        if (re != 0 || im != 0) { buf[w].lab = buf[r].lab; buf[w].re = re; buf[w].im = im; ++w; }
        r = s;
    }
    return w;
}

static int in_sorted(const uint64_t* v, int64_t n, uint64_t x) {
    int64_t lo = 0, hi = n;
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (v[mid] < x) lo = mid + 1; else hi = mid;
    }
    return lo < n && v[lo] == x;
}

static void enum_mon(int M, int p, int pos, int left, int* ex, uint64_t** out, int64_t* n) {
    if (pos == 2 * M) {
        int c[8], a[8];
        for (int m = 0; m < M; ++m) { c[m] = ex[2 * m]; a[m] = ex[2 * m + 1]; }
        for (int t = 0; t < 4; ++t) (*out)[(*n)++] = make_label(t, c, a, M);
        return;
    }
    for (int v = 0; v <= left; ++v) {
        ex[pos] = v;
        enum_mon(M, p, pos + 1, left - v, ex, out, n);
    }
}

/* out[0..5] = N, |E_eta|, NG, |E_L|, |E_C|, 0; returns 0 or -1 on bad input */
int orc_pb_counts(int M, int p, int64_t* out) {
    if (M < 1 || M > 5 || p < 1 || 2 * p > 63) return -1;
    g_M = M;
    int64_t cap = 4 * choose(2 * M + p, p);
    uint64_t* reg = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)cap);
    int64_t N = 0;
    int ex[16];
    enum_mon(M, p, 0, p, ex, &reg, &N);
    qsort(reg, (size_t)N, sizeof(uint64_t), cmp_u64);
    int64_t nd = 0;
    uint64_t* D = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)N);
    uint64_t* OD = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)N);
    int64_t nod = 0;
    for (int64_t r = 0; r < N; ++r) {
        uint64_t L = reg[r];
        int diag = ((L & 3) == 0 || (L & 3) == 3);
        for (int m = 0; m < M; ++m)
            if (expo(L, m, 0) != expo(L, m, 1)) diag = 0;
        if (diag) D[nd++] = L; else OD[nod++] = L;
    }
    const int TCAP = 1 << 16;
    term_t* buf = (term_t*)malloc(sizeof(term_t) * TCAP);
    int64_t eeta = 0, gcap = 1 << 20, ng = 0;
    uint64_t* gen = (uint64_t*)malloc(sizeof(uint64_t) * (size_t)gcap);
    for (int64_t i = 0; i < nd; ++i)
        for (int64_t j = 0; j < nod; ++j) {
            int n = commutator(D[i], OD[j], buf, TCAP);
            if (n < 0) return -1;
            eeta += n;
            for (int t = 0; t < n; ++t) {
                if (ng == gcap) { gcap *= 2; gen = (uint64_t*)realloc(gen, sizeof(uint64_t) * (size_t)gcap); }
                gen[ng++] = buf[t].lab;
            }
        }
    free(buf);
    qsort(gen, (size_t)ng, sizeof(uint64_t), cmp_u64);
    int64_t NG = 0;
    for (int64_t r = 0; r < ng; ++r)
        if (NG == 0 || gen[NG - 1] != gen[r]) gen[NG++] = gen[r];
    int64_t el = 0, ec = 0, bad = 0;
#pragma omp parallel reduction(+ : el, ec, bad)
    {
        term_t* tb = (term_t*)malloc(sizeof(term_t) * TCAP);
#pragma omp for schedule(dynamic, 16)
        for (int64_t a = 0; a < NG; ++a)
            for (int64_t j = 0; j < N; ++j) {
                int n = commutator(gen[a], reg[j], tb, TCAP);
                if (n < 0) { ++bad; continue; }
                for (int t = 0; t < n; ++t) {
                    if (in_sorted(reg, N, tb[t].lab)) ++el; else ++ec;
                }
            }
        free(tb);
    }
    free(reg); free(D); free(OD); free(gen);
    if (bad) return -1;
    out[0] = N; out[1] = eeta; out[2] = NG; out[3] = el; out[4] = ec; out[5] = 0;
    return 0;
}
