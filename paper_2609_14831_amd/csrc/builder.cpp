// Graph compiler and bundle I/O (host).
//
// Compilation follows Sec. 2.3 of the paper: two deterministic traversals of
// the same algebra.  Traversal 1 counts the records of every target, which
// fixes the exact length of every on-disk array; the bundle file is then sized
// and memory-mapped; traversal 2 regenerates the algebra and writes each record
// directly into its final slot.  Peak memory is the registry plus one target's
// local expansion per thread -- no graph-sized intermediate.
//
// Algebras (registry order is the external index space):
//  * E_pq over n orbitals, index p*n+q, [E_pq, E_rs] = d_qr E_ps - d_ps E_rq.
//  * Even Majorana strings of degree 2 and 4 over m modes, 2-subsets then
//    4-subsets in lexicographic order; basis Gamma_S = i^{d(d-1)/2} gamma_S,
//    generator basis i*Gamma_S; projection keeps degree <= 4 (Eq. projected-flow).
//    A target collects every ordered pair (A, B) of anticommuting strings with
//    A xor B = target; the factor c of [i Gamma_A, Gamma_B] = c Gamma_{A xor B}
//    is +-2.
#include <fcntl.h>
#include <sys/mman.h>
#include <sys/stat.h>
#include <unistd.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <functional>
#include <thread>
#include <unordered_map>

#include "internal.h"

namespace cut {

// ------------------------------------------------------------- checksum ----
// 64-bit checksum: independent 1 MiB chunks hashed word by word (multiply-xor
// mixing), chunk digests folded in order.  Deterministic for any thread count.
static inline uint64_t mix64(uint64_t x) {
    x ^= x >> 31;
    x *= 0x7fb5d329728ea185ull;
    x ^= x >> 27;
    x *= 0x81dadef4bc2dd44dull;
    x ^= x >> 33;
    return x;
}

static uint64_t chunk_hash(const uint8_t* p, uint64_t n, uint64_t seed) {
    uint64_t h = seed ^ (n * 0x9e3779b97f4a7c15ull);
    uint64_t w = 0;
    uint64_t i = 0;
    for (; i + 8 <= n; i += 8) {
        std::memcpy(&w, p + i, 8);
        h = (h ^ mix64(w + i)) * 0x100000001b3ull;
    }
    uint64_t tail = 0;
    for (uint64_t t = 0; i < n; ++i, ++t) tail |= (uint64_t)p[i] << (8 * t);
    h = (h ^ mix64(tail ^ 0xabcdefull)) * 0x100000001b3ull;
    return mix64(h);
}

uint64_t checksum64(const void* data, uint64_t bytes) {
    const uint64_t C = 1ull << 20;
    const uint64_t nchunk = (bytes + C - 1) / C;
    std::vector<uint64_t> dig(nchunk ? nchunk : 1, 0);
    unsigned nt = std::max(1u, std::min<unsigned>(std::thread::hardware_concurrency(), 16));
    std::atomic<uint64_t> next{0};
    auto work = [&]() {
        for (uint64_t c; (c = next.fetch_add(1)) < nchunk;) {
            uint64_t b = c * C, n = std::min(C, bytes - b);
            dig[c] = chunk_hash((const uint8_t*)data + b, n, c);
        }
    };
    std::vector<std::thread> th;
    for (unsigned t = 1; t < nt && nchunk > 1; ++t) th.emplace_back(work);
    work();
    for (auto& t : th) t.join();
    uint64_t h = 0x243f6a8885a308d3ull ^ bytes;
    for (uint64_t d : dig) h = mix64(h ^ d) + 0x9e3779b97f4a7c15ull;
    return h;
}

// ------------------------------------------------------------- algebras ----
struct Rec {
    int32_t i, j;
    int8_t c;
};

// Lexicographic rank of an r-subset {c_1 < ... < c_r} of [0, m), by the
// hockey-stick identity: sum_t [C(m-c_{t-1}-1, r-t+1) - C(m-c_t, r-t+1)], c_0 = -1.
struct Ranker {
    int m;
    int64_t binom[66][6];
    int64_t nquad;
    explicit Ranker(int m_) : m(m_) {
        for (int a = 0; a <= 65; ++a)
            for (int b = 0; b <= 5; ++b) {
                if (b == 0) binom[a][b] = 1;
                else if (a == 0) binom[a][b] = 0;
                else binom[a][b] = binom[a - 1][b - 1] + binom[a - 1][b];
            }
        nquad = binom[m][2];
    }
    int64_t C(int a, int b) const { return (a < 0 || b < 0) ? 0 : binom[a][b]; }
    int64_t rank(uint64_t mask) const {
        int elems[4];
        int r = 0;
        for (uint64_t x = mask; x; x &= x - 1) elems[r++] = __builtin_ctzll(x);
        int64_t v = 0;
        int prev = -1;
        for (int t = 0; t < r; ++t) {
            v += C(m - prev - 1, r - t) - C(m - elems[t], r - t);
            prev = elems[t];
        }
        return r == 2 ? v : nquad + v;
    }
};

// Sign of [i Gamma_A, Gamma_B] for anticommuting even strings.  Reordering
// gamma_A gamma_B into ascending order costs (-1)^{#(a,b): a>b}; its parity is
// popcount(A & M) mod 2 where bit p of M is the parity of #{b in B : b < p}
// (a prefix xor of B shifted up by one).  Phases i^{d(d-1)/2} of the three
// strings and the factor 2i of the anticommutator complete c = 2 i^e.
static inline int8_t maj_factor(uint64_t A, uint64_t B) {
    uint64_t M = B << 1;
    M ^= M << 1;
    M ^= M << 2;
    M ^= M << 4;
    M ^= M << 8;
    M ^= M << 16;
    M ^= M << 32;
    int par = __builtin_popcountll(A & M) & 1;
    auto tri = [](int d) { return (d * (d - 1) / 2) & 3; };
    int e = 1 + tri(__builtin_popcountll(A)) + tri(__builtin_popcountll(B)) -
            tri(__builtin_popcountll(A ^ B)) + 2 * par;
    e &= 3;
    return e == 0 ? 2 : -2;  // e is even for anticommuting Hermitian strings
}

struct Algebra {
    int kind, size;
    int64_t N;
    std::vector<uint64_t> labels;
    std::vector<uint8_t> diag;
    std::vector<int32_t> pairs;
    int gen_sign;
    Ranker rk;
    Algebra(int kind_, int size_) : kind(kind_), size(size_), rk(kind_ == CUT_ALG_MAJORANA ? size_ : 4) {
        if (kind == CUT_ALG_EPQ) {
            int n = size;
            N = (int64_t)n * n;
            for (int p = 0; p < n; ++p)
                for (int q = 0; q < n; ++q) {
                    labels.push_back(((uint64_t)p << 32) | (uint64_t)q);
                    diag.push_back(p == q);
                }
            for (int p = 0; p < n; ++p) pairs.push_back(p * n + p);
            gen_sign = 1;
        } else {
            int m = size;
            for (int a = 0; a < m; ++a)
                for (int b = a + 1; b < m; ++b) labels.push_back((1ull << a) | (1ull << b));
            for (int a = 0; a < m; ++a)
                for (int b = a + 1; b < m; ++b)
                    for (int c = b + 1; c < m; ++c)
                        for (int d = c + 1; d < m; ++d)
                            labels.push_back((1ull << a) | (1ull << b) | (1ull << c) | (1ull << d));
            N = (int64_t)labels.size();
            const uint64_t even = 0x5555555555555555ull;
            for (uint64_t L : labels) diag.push_back((L & even) == ((L >> 1) & even));
            for (int a = 0; a < m / 2; ++a) pairs.push_back((int32_t)rk.rank((3ull << (2 * a))));
            gen_sign = -1;
        }
    }

    // Expands every record of target k into out (unsorted).
    void expand(int64_t k, std::vector<Rec>& out) const {
        out.clear();
        if (kind == CUT_ALG_EPQ) {
            const int n = size;
            const int a = (int)(k / n), b = (int)(k % n);
            // [E_aq, E_qb] contributes +E_ab; [E_pb, E_ap] contributes -E_ab
            for (int q = 0; q < n; ++q) out.push_back({a * n + q, q * n + b, 1});
            for (int p = 0; p < n; ++p) out.push_back({p * n + b, a * n + p, -1});
            // merge equal (i, j) and drop zero factors
            std::sort(out.begin(), out.end(), [](const Rec& x, const Rec& y) {
                return x.i != y.i ? x.i < y.i : x.j < y.j;
            });
            size_t w = 0;
            for (size_t r = 0; r < out.size();) {
                size_t s = r;
                int sum = 0;
                while (s < out.size() && out[s].i == out[r].i && out[s].j == out[r].j) sum += out[s++].c;
                if (sum != 0) out[w++] = {out[r].i, out[r].j, (int8_t)sum};
                r = s;
            }
            out.resize(w);
            return;
        }
        const int m = size;
        const uint64_t K = labels[(size_t)k];
        const uint64_t full = (m == 64) ? ~0ull : ((1ull << m) - 1);
        auto emit = [&](uint64_t A, uint64_t B) {
            out.push_back({(int32_t)rk.rank(A), (int32_t)rk.rank(B), maj_factor(A, B)});
        };
        if (__builtin_popcountll(K) == 2) {
            const int a = __builtin_ctzll(K), b = 63 - __builtin_clzll(K);
            const uint64_t rest = full & ~K;
            // quadratic x quadratic sharing one mode
            for (uint64_t x = rest; x; x &= x - 1) {
                uint64_t c = x & (~x + 1);
                emit((1ull << a) | c, (1ull << b) | c);
                emit((1ull << b) | c, (1ull << a) | c);
            }
            // quartic x quartic sharing three modes
            for (uint64_t x1 = rest; x1; x1 &= x1 - 1) {
                uint64_t t1 = x1 & (~x1 + 1);
                for (uint64_t x2 = x1 & (x1 - 1); x2; x2 &= x2 - 1) {
                    uint64_t t2 = x2 & (~x2 + 1);
                    for (uint64_t x3 = x2 & (x2 - 1); x3; x3 &= x3 - 1) {
                        uint64_t T = t1 | t2 | (x3 & (~x3 + 1));
                        emit(T | (1ull << a), T | (1ull << b));
                        emit(T | (1ull << b), T | (1ull << a));
                    }
                }
            }
        } else {
            // quadratic {p,q} with p in K, q not in K, against the quartic K^{p,q}
            for (uint64_t xp = K; xp; xp &= xp - 1) {
                uint64_t p = xp & (~xp + 1);
                for (uint64_t xq = full & ~K; xq; xq &= xq - 1) {
                    uint64_t q = xq & (~xq + 1);
                    uint64_t Q = p | q, F = K ^ Q;
                    emit(Q, F);
                    emit(F, Q);
                }
            }
        }
        std::sort(out.begin(), out.end(),
                  [](const Rec& x, const Rec& y) { return x.i != y.i ? x.i < y.i : x.j < y.j; });
    }

    // Outside registry of a Majorana graph: every 6-subset of the modes,
    // lexicographic (the degree-6 strings [eta, X] reaches outside the
    // degree <= 4 registry, Eq. projected-flow).
    std::vector<uint64_t> outside_labels() const {
        std::vector<uint64_t> out;
        const int m = size;
        int c[6] = {0, 1, 2, 3, 4, 5};
        if (m < 6) return out;
        for (;;) {
            uint64_t L = 0;
            for (int t = 0; t < 6; ++t) L |= 1ull << c[t];
            out.push_back(L);
            int t = 5;
            while (t >= 0 && c[t] == m - 6 + t) --t;
            if (t < 0) break;
            ++c[t];
            for (int u = t + 1; u < 6; ++u) c[u] = c[u - 1] + 1;
        }
        return out;
    }

    // Records of outside target Q (degree 6): [i Gamma_A, Gamma_B] has a
    // degree-6 part only for two quartics sharing one mode, so A = T1 + s and
    // B = T2 + s for an ordered split of Q into triples (T1, T2) and a mode s
    // outside Q.  Sorted by (i, j).
    void expand_outside(uint64_t Q, std::vector<Rec>& out) const {
        out.clear();
        const int m = size;
        const uint64_t full = (m == 64) ? ~0ull : ((1ull << m) - 1);
        int q[6], n = 0;
        for (uint64_t x = Q; x; x &= x - 1) q[n++] = __builtin_ctzll(x);
        for (int a = 0; a < 6; ++a)
            for (int b = a + 1; b < 6; ++b)
                for (int c = b + 1; c < 6; ++c) {
                    const uint64_t T1 = (1ull << q[a]) | (1ull << q[b]) | (1ull << q[c]);
                    const uint64_t T2 = Q ^ T1;
                    for (uint64_t xs = full & ~Q; xs; xs &= xs - 1) {
                        const uint64_t sbit = xs & (~xs + 1);
                        const uint64_t A = T1 | sbit, B = T2 | sbit;
                        out.push_back({(int32_t)rk.rank(A), (int32_t)rk.rank(B), maj_factor(A, B)});
                    }
                }
        std::sort(out.begin(), out.end(),
                  [](const Rec& x, const Rec& y) { return x.i != y.i ? x.i < y.i : x.j < y.j; });
    }

    std::string identifier() const {
        char buf[96];
        if (kind == CUT_ALG_EPQ)
            snprintf(buf, sizeof buf, "epq n=%d order=p*n+q gen=E_pq factors=int8", size);
        else
            snprintf(buf, sizeof buf, "majorana m=%d deg=2,4 order=lex2,lex4 proj=deg<=4 gen=iGamma factors=int8",
                     size);
        return buf;
    }
};

// ---------------------------------------------------------------- writer ----
static uint64_t align64(uint64_t x) { return (x + 63) & ~uint64_t(63); }

static void parallel_for(int64_t n, int threads, const std::function<void(int64_t, int64_t)>& fn) {
    int nt = std::max(1, threads);
    if (n < 4096 || nt == 1) {
        fn(0, n);
        return;
    }
    std::atomic<int64_t> next{0};
    const int64_t blk = 512;
    auto work = [&]() {
        for (int64_t b; (b = next.fetch_add(blk)) < n;) fn(b, std::min(n, b + blk));
    };
    std::vector<std::thread> th;
    for (int t = 1; t < nt; ++t) th.emplace_back(work);
    work();
    for (auto& t : th) t.join();
}


// ------------------------------------------------------------ Pauli-boson --
// Labels B_{tau,c,a} = sigma_tau prod_m (b_m^+)^{c_m} b_m^{a_m} (Eq. monomial),
// each packed into one 64-bit key whose numeric order is the canonical order
// (total bosonic degree, tau, c_1, a_1, ..., c_M, a_M): W bits per field, the
// degree on top, then tau (2 bits), then the exponents, c_1 most significant.
// W holds 3p, the largest exponent or degree a commutator of a generator label
// (degree <= 2p) with a registry label (degree <= p) can reach.
struct PBCodec {
    int M = 0, W = 0;
    uint64_t key(int tau, const int* c, const int* a) const {
        uint64_t d = 0, v = 0;
        for (int m = 0; m < M; ++m) {
            d += (uint64_t)(c[m] + a[m]);
            v = (v << W) | (uint64_t)c[m];
            v = (v << W) | (uint64_t)a[m];
        }
        return (((d << 2) | (uint64_t)tau) << (2 * M * W)) | v;
    }
    void unpack(uint64_t k, int& tau, int* c, int* a) const {
        const uint64_t mask = (1ull << W) - 1;
        for (int m = M - 1; m >= 0; --m) {
            a[m] = (int)(k & mask);
            k >>= W;
            c[m] = (int)(k & mask);
            k >>= W;
        }
        tau = (int)(k & 3);
    }
};

// Factors are exact 128-bit Gaussian integers: normal ordering of the degree-24
// one-mode registry reaches 24! C(48, 24) ~ 2e37, beyond int64.
typedef __int128 i128;

struct PBTerm {
    uint64_t key;
    i128 re, im;
};

// [B_A, B_B] = B_A B_B - B_B B_A, merged by label, zero sums dropped.  Pauli
// part: sigma_t sigma_u = i^e sigma_w (x y = i z and cyclic); boson part per
// mode: (b^+)^c1 b^a1 (b^+)^c2 b^a2 = sum_k k! C(a1,k) C(c2,k) (b^+)^(c1+c2-k)
// b^(a1+a2-k) (each of k annihilators of the left factor contracted with a
// creator of the right one).
struct PBAlgebra {
    PBCodec cd;
    int p = 0;
    int64_t binom[64][64];                      // C(63, 31) < 2^63
    i128 fact[34];                              // 33! < 2^127
    PBAlgebra(int M_, int p_) : p(p_) {
        cd.M = M_;
        int w = 1;
        while ((1 << w) <= 3 * p_) ++w;
        cd.W = w;
        for (int n = 0; n < 64; ++n)
            for (int k = 0; k < 64; ++k) binom[n][k] = (k == 0) ? 1 : (n == 0 ? 0 : binom[n - 1][k - 1] + binom[n - 1][k]);
        fact[0] = 1;
        for (int n = 1; n < 34; ++n) fact[n] = fact[n - 1] * n;
    }
    // 64-bit labels; a product's exponents (<= 2p) index binom and its
    // contraction orders (<= p, one factor is a registry label) index fact
    bool fits() const { return (2 * cd.M + 1) * cd.W + 2 <= 64 && 2 * p < 64; }
    mutable std::atomic<bool> overflow{false};   // a factor left the int128 range (never cleared)

    static void pauli(int t, int u, int& w, int& e) {
        if (t == 0 || u == 0) {
            w = t + u;
            e = 0;
        } else if (t == u) {
            w = 0;
            e = 0;
        } else {
            w = 6 - t - u;
            e = ((t == 1 && u == 2) || (t == 2 && u == 3) || (t == 3 && u == 1)) ? 1 : 3;
        }
    }
    // appends sign * B_X B_Y
    void product(uint64_t X, uint64_t Y, int sign, std::vector<PBTerm>& out) const {
        const int M = cd.M;
        int tx, ty, cx[8], ax[8], cy[8], ay[8];
        cd.unpack(X, tx, cx, ax);
        cd.unpack(Y, ty, cy, ay);
        int w, e;
        pauli(tx, ty, w, e);
        static const int ere[4] = {1, 0, -1, 0}, eim[4] = {0, 1, 0, -1};
        int k[8] = {0}, kmax[8], c[8], a[8];
        for (int m = 0; m < M; ++m) kmax[m] = std::min(ax[m], cy[m]);
        for (;;) {
            // the factor in 64-bit arithmetic while it fits (every registry
            // but the highest-degree ones), else again in 128-bit
            int64_t f64 = sign;
            bool wide = false;
            for (int m = 0; m < M && !wide; ++m) {
                int64_t g;
                wide = k[m] > 20 || __builtin_mul_overflow((int64_t)fact[k[m]], binom[ax[m]][k[m]], &g) ||
                       __builtin_mul_overflow(g, binom[cy[m]][k[m]], &g) || __builtin_mul_overflow(f64, g, &f64);
            }
            i128 f = f64;
            if (wide) {
                f = sign;
                for (int m = 0; m < M; ++m) {
                    i128 g;
                    if (__builtin_mul_overflow(fact[k[m]], (i128)binom[ax[m]][k[m]], &g) ||
                        __builtin_mul_overflow(g, (i128)binom[cy[m]][k[m]], &g) || __builtin_mul_overflow(f, g, &f))
                        overflow = true;
                }
            }
            for (int m = 0; m < M; ++m) {
                c[m] = cx[m] + cy[m] - k[m];
                a[m] = ax[m] + ay[m] - k[m];
            }
            out.push_back({cd.key(w, c, a), ere[e] * f, eim[e] * f});
            int m = 0;
            while (m < M && k[m] == kmax[m]) k[m++] = 0;
            if (m == M) break;
            ++k[m];
        }
    }
    void commutator(uint64_t A, uint64_t B, std::vector<PBTerm>& out) const {
        out.clear();
        product(A, B, 1, out);
        product(B, A, -1, out);
        std::sort(out.begin(), out.end(), [](const PBTerm& x, const PBTerm& y) { return x.key < y.key; });
        size_t w = 0;
        for (size_t r = 0; r < out.size();) {
            size_t s = r;
            i128 re = 0, im = 0;
            for (; s < out.size() && out[s].key == out[r].key; ++s)
                if (__builtin_add_overflow(re, out[s].re, &re) || __builtin_add_overflow(im, out[s].im, &im))
                    overflow = true;
            if (re != 0 || im != 0) out[w++] = {out[r].key, re, im};
            r = s;
        }
        out.resize(w);
    }
    // the complete degree-p registry, canonical order
    std::vector<uint64_t> registry() const {
        std::vector<uint64_t> out;
        const int M = cd.M;
        std::vector<int> ex(2 * M, 0);
        std::function<void(int, int)> rec = [&](int pos, int left) {
            if (pos == 2 * M) {
                int c[8], a[8];
                for (int m = 0; m < M; ++m) {
                    c[m] = ex[2 * m];
                    a[m] = ex[2 * m + 1];
                }
                for (int t = 0; t < 4; ++t) out.push_back(cd.key(t, c, a));
                return;
            }
            for (int v = 0; v <= left; ++v) {
                ex[pos] = v;
                rec(pos + 1, left - v);
            }
        };
        rec(0, p);
        std::sort(out.begin(), out.end());
        return out;
    }
    bool diagonal(uint64_t L) const {
        int t, c[8], a[8];
        cd.unpack(L, t, c, a);
        if (t != 0 && t != 3) return false;
        for (int m = 0; m < cd.M; ++m)
            if (c[m] != a[m]) return false;
        return true;
    }
};

template <class F>
struct PBRec {
    int32_t i, j;
    F re, im;
};

// sorts every segment [off[s], off[s+1]) of the arrays (ri, rj, rc) by (ri, rj);
// rc holds (re, im) pairs of F
template <class F>
static void sort_segments(const std::vector<int64_t>& off, int32_t* ri, int32_t* rj, F* rc, int nt) {
    const int64_t nseg = (int64_t)off.size() - 1;
    parallel_for(nseg, nt, [&](int64_t b, int64_t e) {
        std::vector<PBRec<F>> tmp;
        for (int64_t s = b; s < e; ++s) {
            const int64_t o = off[s], n = off[s + 1] - off[s];
            tmp.resize((size_t)n);
            for (int64_t t = 0; t < n; ++t) tmp[t] = {ri[o + t], rj[o + t], rc[2 * (o + t)], rc[2 * (o + t) + 1]};
            std::sort(tmp.begin(), tmp.end(),
                      [](const PBRec<F>& x, const PBRec<F>& y) { return x.i != y.i ? x.i < y.i : x.j < y.j; });
            for (int64_t t = 0; t < n; ++t) {
                ri[o + t] = tmp[t].i;
                rj[o + t] = tmp[t].j;
                rc[2 * (o + t)] = tmp[t].re;
                rc[2 * (o + t) + 1] = tmp[t].im;
            }
        }
    });
}

static bool fits_i16(i128 v) { return v >= -32767 && v <= 32767; }

// Factor arrays of a Pauli-boson bundle: (re, im) pairs of int16 while every
// factor fits (4 bytes a record), else of FP64 (16 bytes a record, each factor
// the FP64 value nearest the exact integer).
struct PBFactors {
    uint8_t* base = nullptr;
    bool wide = false;
    void put(int64_t q, i128 re, i128 im) const {
        if (wide) {
            const double v[2] = {(double)re, (double)im};
            std::memcpy(base + 16 * q, v, 16);
        } else {
            const int16_t v[2] = {(int16_t)re, (int16_t)im};
            std::memcpy(base + 4 * q, v, 4);
        }
    }
};

// Compiles the Pauli-boson graph (Sec. 2.2-2.3): registry, generator records
// E_eta and generator registry, retained records E_L and (optionally) the
// outside-space records E_C, product-major in two traversals over the pairs
// (generator label, registry label): the first counts the records of every
// target (and collects the outside labels), the exact-size file is mapped, the
// second writes each record at a per-target cursor, and every segment is then
// sorted by (left, right) input so the bytes do not depend on the thread count.
static cut_status build_pauli_boson(int M, int p, const char* path, int nt, bool outside, cut_graph_desc* desc) {
    int fd = -1;
    void* map = MAP_FAILED;
    size_t map_bytes = 0;
    try {
        auto t0 = std::chrono::steady_clock::now();
        PBAlgebra alg(M, p);
        if (!alg.fits()) CUT_FAIL(CUT_E_UNSUPPORTED, "cut_graph_build: Pauli-boson M=%d p=%d too large for 64-bit labels", M, p);
        const std::vector<uint64_t> reg = alg.registry();
        const int64_t N = (int64_t)reg.size();
        if (N >= (1ll << 23)) CUT_FAIL(CUT_E_UNSUPPORTED, "cut_graph_build: registry of %lld labels", (long long)N);
        std::unordered_map<uint64_t, int32_t> ridx;
        ridx.reserve((size_t)N * 2);
        for (int64_t r = 0; r < N; ++r) ridx[reg[(size_t)r]] = (int32_t)r;
        std::vector<uint8_t> diag((size_t)N);
        std::vector<int32_t> D, OD;
        for (int64_t r = 0; r < N; ++r) {
            diag[(size_t)r] = alg.diagonal(reg[(size_t)r]) ? 1 : 0;
            (diag[(size_t)r] ? D : OD).push_back((int32_t)r);
        }
        // generator: [B_i, B_j], i diagonal, j not; its labels form the generator registry
        struct GRec {
            uint64_t key;
            int32_t i, j;
            i128 re, im;
        };
        std::vector<GRec> graw;
        std::atomic<int> wide{0};          // a factor leaves int16: FP64 factor arrays
        {
            std::vector<PBTerm> t;
            for (int32_t i : D)
                for (int32_t j : OD) {
                    alg.commutator(reg[(size_t)i], reg[(size_t)j], t);
                    for (auto& x : t) {
                        graw.push_back({x.key, i, j, x.re, x.im});
                        if (!fits_i16(x.re) || !fits_i16(x.im)) wide = 1;
                    }
                }
        }
        std::vector<uint64_t> gen;
        gen.reserve(graw.size());
        for (auto& r : graw) gen.push_back(r.key);
        std::sort(gen.begin(), gen.end());
        gen.erase(std::unique(gen.begin(), gen.end()), gen.end());
        const int64_t NG = (int64_t)gen.size();
        if (NG >= (1ll << 23)) CUT_FAIL(CUT_E_UNSUPPORTED, "cut_graph_build: generator registry of %lld labels", (long long)NG);
        std::unordered_map<uint64_t, int32_t> gidx;
        gidx.reserve((size_t)NG * 2);
        for (int64_t r = 0; r < NG; ++r) gidx[gen[(size_t)r]] = (int32_t)r;
        std::sort(graw.begin(), graw.end(), [&](const GRec& x, const GRec& y) {
            const int32_t ax = gidx[x.key], ay = gidx[y.key];
            return ax != ay ? ax < ay : (x.i != y.i ? x.i < y.i : x.j < y.j);
        });
        const int64_t Eg = (int64_t)graw.size();
        std::vector<int64_t> goff((size_t)NG + 1, 0);
        for (auto& r : graw) goff[(size_t)gidx[r.key] + 1]++;
        for (int64_t a = 0; a < NG; ++a) goff[a + 1] += goff[a];

        // candidate outside labels: every label of degree p+1 .. 3p (a bracket of a
        // generator label, degree <= 2p, with a registry label reaches no
        // further), indexed once; the outside registry is the subset reached
        std::vector<uint64_t> cand;
        std::unordered_map<uint64_t, int32_t> cidx;
        if (outside) {
            PBAlgebra wide(M, 3 * p);
            wide.cd = alg.cd;                       // same key layout
            for (uint64_t key : wide.registry())
                if (!ridx.count(key)) cand.push_back(key);
            if ((int64_t)cand.size() >= (1ll << 31)) CUT_FAIL(CUT_E_UNSUPPORTED, "cut_graph_build: outside space too large");
            cidx.reserve(cand.size() * 2);
            for (size_t q = 0; q < cand.size(); ++q) cidx[cand[q]] = (int32_t)q;
        }
        // traversal 1: counts per retained target and per candidate outside label
        std::vector<std::vector<int64_t>> tcnt(nt, std::vector<int64_t>((size_t)N, 0));
        std::vector<std::atomic<int64_t>> ccnt(cand.size());
        for (auto& c : ccnt) c.store(0, std::memory_order_relaxed);
        {
            std::atomic<int64_t> next{0};
            std::atomic<int> stray{0};
            auto work = [&](int tid) {
                std::vector<PBTerm> t;
                for (int64_t a; (a = next.fetch_add(1)) < NG;)
                    for (int64_t j = 0; j < N; ++j) {
                        alg.commutator(gen[(size_t)a], reg[(size_t)j], t);
                        for (auto& x : t) {
                            auto it = ridx.find(x.key);
                            const bool w16 = !fits_i16(x.re) || !fits_i16(x.im);
                            if (it != ridx.end()) {
                                tcnt[tid][(size_t)it->second]++;
                                if (w16) wide = 1;
                            } else if (outside) {
                                if (w16) wide = 1;
                                auto ic = cidx.find(x.key);
                                if (ic == cidx.end()) stray = 1;
                                else ccnt[(size_t)ic->second].fetch_add(1, std::memory_order_relaxed);
                            }
                        }
                    }
            };
            std::vector<std::thread> th;
            for (int q = 1; q < nt; ++q) th.emplace_back(work, q);
            work(0);
            for (auto& x : th) x.join();
            if (stray) CUT_FAIL(CUT_E_UNSUPPORTED, "cut_graph_build: a bracket left the degree-3p label space");
        }
        std::vector<int64_t> loff((size_t)N + 1, 0);
        for (int q = 0; q < nt; ++q)
            for (int64_t k = 0; k < N; ++k) loff[k + 1] += tcnt[q][(size_t)k];
        tcnt.clear();
        for (int64_t k = 0; k < N; ++k) loff[k + 1] += loff[k];
        const int64_t E = loff[(size_t)N];
        std::vector<uint64_t> olab;
        std::vector<int64_t> coff(1, 0);
        std::vector<int32_t> cand2out(cand.size(), -1);   // candidate -> outside registry index
        for (size_t q = 0; q < cand.size(); ++q) {
            const int64_t n = ccnt[q].load(std::memory_order_relaxed);
            if (n == 0) continue;
            cand2out[q] = (int32_t)olab.size();
            olab.push_back(cand[q]);
            coff.push_back(coff.back() + n);
        }
        ccnt = std::vector<std::atomic<int64_t>>();
        const int64_t Nc = (int64_t)olab.size(), Ec = coff.back();
        if (alg.overflow) CUT_FAIL(CUT_E_UNSUPPORTED, "cut_graph_build: a factor exceeds the int128 range");
        const uint32_t fb = wide ? 16 : 4;

        // file layout: base sections, generator labels, outside sections
        struct Sz {
            uint32_t id, eb;
            uint64_t count;
        };
        std::vector<Sz> secs = {{SEC_LABELS, 8, (uint64_t)N},       {SEC_DIAG, 1, (uint64_t)N},
                                {SEC_PAIRS, 4, 0},                   {SEC_FLOW_OFF, 8, (uint64_t)N + 1},
                                {SEC_FLOW_I, 4, (uint64_t)E},        {SEC_FLOW_J, 4, (uint64_t)E},
                                {SEC_FLOW_C, fb, (uint64_t)E},       {SEC_GEN_OFF, 8, (uint64_t)NG + 1},
                                {SEC_GEN_I, 4, (uint64_t)Eg},        {SEC_GEN_J, 4, (uint64_t)Eg},
                                {SEC_GEN_C, fb, (uint64_t)Eg},       {SEC_GEN_LABELS, 8, (uint64_t)NG}};
        if (outside) {
            secs.push_back({SEC_OUT_LABELS, 8, (uint64_t)Nc});
            secs.push_back({SEC_OUT_OFF, 8, (uint64_t)Nc + 1});
            secs.push_back({SEC_OUT_I, 4, (uint64_t)Ec});
            secs.push_back({SEC_OUT_J, 4, (uint64_t)Ec});
            secs.push_back({SEC_OUT_C, fb, (uint64_t)Ec});
        }
        const int nsec = (int)secs.size();
        SectionEntry tab[kMaxSections];
        const size_t tab_bytes = nsec * sizeof(SectionEntry);
        uint64_t pos = align64(sizeof(BundleHeader) + tab_bytes);
        for (int s = 0; s < nsec; ++s) {
            tab[s] = {secs[s].id, secs[s].eb, pos, secs[s].count, 0};
            pos = align64(pos + secs[s].count * secs[s].eb);
        }
        const uint64_t file_bytes = pos;
        std::string tmp = std::string(path) + ".tmp";
        fd = ::open(tmp.c_str(), O_RDWR | O_CREAT | O_TRUNC, 0644);
        if (fd < 0) CUT_FAIL(CUT_E_IO, "cannot create %s", tmp.c_str());
        if (::ftruncate(fd, (off_t)file_bytes) != 0) CUT_FAIL(CUT_E_IO, "cannot size %s", tmp.c_str());
        map = ::mmap(nullptr, file_bytes, PROT_READ | PROT_WRITE, MAP_SHARED, fd, 0);
        if (map == MAP_FAILED) CUT_FAIL(CUT_E_IO, "cannot map %s", tmp.c_str());
        map_bytes = file_bytes;
        uint8_t* base = (uint8_t*)map;
        auto sec = [&](int s) { return base + tab[s].offset; };
        std::memcpy(sec(0), reg.data(), N * 8);
        std::memcpy(sec(1), diag.data(), N);
        std::memcpy(sec(3), loff.data(), (N + 1) * 8);
        std::memcpy(sec(7), goff.data(), (NG + 1) * 8);
        std::memcpy(sec(11), gen.data(), NG * 8);
        {
            int32_t* Gi = (int32_t*)sec(8);
            int32_t* Gj = (int32_t*)sec(9);
            const PBFactors Gc{sec(10), fb == 16};
            for (int64_t e = 0; e < Eg; ++e) {
                Gi[e] = graw[(size_t)e].i;
                Gj[e] = graw[(size_t)e].j;
                Gc.put(e, graw[(size_t)e].re, graw[(size_t)e].im);
            }
        }
        graw.clear();
        graw.shrink_to_fit();
        int32_t* Li = (int32_t*)sec(4);
        int32_t* Lj = (int32_t*)sec(5);
        const PBFactors Lc{sec(6), fb == 16};
        int32_t* Ci = outside ? (int32_t*)sec(14) : nullptr;
        int32_t* Cj = outside ? (int32_t*)sec(15) : nullptr;
        const PBFactors Cc{outside ? sec(16) : nullptr, fb == 16};
        if (outside) {
            std::memcpy(sec(12), olab.data(), Nc * 8);
            std::memcpy(sec(13), coff.data(), (Nc + 1) * 8);
        }
        // traversal 2: every record at its target's cursor
        {
            std::vector<std::atomic<int64_t>> curL((size_t)N), curC((size_t)Nc);
            for (int64_t k = 0; k < N; ++k) curL[(size_t)k] = loff[(size_t)k];
            for (int64_t q = 0; q < Nc; ++q) curC[(size_t)q] = coff[(size_t)q];
            std::atomic<int64_t> next{0};
            auto work = [&]() {
                std::vector<PBTerm> t;
                for (int64_t a; (a = next.fetch_add(1)) < NG;)
                    for (int64_t j = 0; j < N; ++j) {
                        alg.commutator(gen[(size_t)a], reg[(size_t)j], t);
                        for (auto& x : t) {
                            auto it = ridx.find(x.key);
                            if (it != ridx.end()) {
                                const int64_t q = curL[(size_t)it->second].fetch_add(1);
                                Li[q] = (int32_t)a;
                                Lj[q] = (int32_t)j;
                                Lc.put(q, x.re, x.im);
                            } else if (outside) {
                                const int64_t q = curC[(size_t)cand2out[(size_t)cidx.at(x.key)]].fetch_add(1);
                                Ci[q] = (int32_t)a;
                                Cj[q] = (int32_t)j;
                                Cc.put(q, x.re, x.im);
                            }
                        }
                    }
            };
            std::vector<std::thread> th;
            for (int q = 1; q < nt; ++q) th.emplace_back(work);
            work();
            for (auto& x : th) x.join();
        }
        if (fb == 16) {
            sort_segments(loff, Li, Lj, (double*)Lc.base, nt);
            if (outside) sort_segments(coff, Ci, Cj, (double*)Cc.base, nt);
        } else {
            sort_segments(loff, Li, Lj, (int16_t*)Lc.base, nt);
            if (outside) sort_segments(coff, Ci, Cj, (int16_t*)Cc.base, nt);
        }

        for (int s = 0; s < nsec; ++s) tab[s].checksum = checksum64(sec(s), tab[s].count * tab[s].elem_bytes);
        BundleHeader h{};
        std::memcpy(h.magic, kMagic, 8);
        h.version = kVersion;
        h.header_bytes = sizeof(BundleHeader);
        h.algebra = CUT_ALG_PAULI_BOSON;
        h.size = 256 * M + p;
        h.n_ops = N;
        h.n_records = E;
        h.n_gen_records = Eg;
        h.n_pairs = 0;
        h.factor_bytes = (int32_t)fb;
        h.gen_sign = 1;
        h.n_sections = (uint32_t)nsec;
        h.section_table_offset = sizeof(BundleHeader);
        h.file_bytes = file_bytes;
        h.n_out_ops = Nc;
        h.n_out_records = Ec;
        h.n_gen_ops = NG;
        uint64_t rc = 0;
        for (int s = 3; s < nsec; ++s) rc = mix64(rc ^ tab[s].checksum);
        h.records_checksum = rc;
        snprintf(h.identifier, sizeof h.identifier,
                 "pauli-boson M=%d p=%d key=deg,tau,c1,a1..:%d bits order=key mask=I|z,c=a factors=%s", M, p,
                 alg.cd.W, fb == 16 ? "f64x2" : "int16x2");
        h.header_checksum = 0;
        std::memcpy(base + sizeof(BundleHeader), tab, tab_bytes);
        h.header_checksum = checksum64(&h, sizeof h) ^ checksum64(tab, tab_bytes);
        std::memcpy(base, &h, sizeof h);
        if (::msync(map, map_bytes, MS_SYNC) != 0) CUT_FAIL(CUT_E_IO, "msync failed");
        ::munmap(map, map_bytes);
        map = MAP_FAILED;
        ::close(fd);
        fd = -1;
        if (::rename(tmp.c_str(), path) != 0) CUT_FAIL(CUT_E_IO, "cannot rename %s to %s", tmp.c_str(), path);
        if (desc) {
            std::memset(desc, 0, sizeof *desc);
            desc->algebra = CUT_ALG_PAULI_BOSON;
            desc->size = h.size;
            desc->n_ops = N;
            desc->n_records = E;
            desc->n_gen_records = Eg;
            desc->n_pairs = 0;
            desc->n_out_ops = Nc;
            desc->n_out_records = Ec;
            desc->n_gen_ops = NG;
            desc->checksum = rc;
            desc->file_bytes = (int64_t)file_bytes;
            desc->build_seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            std::strncpy(desc->identifier, h.identifier, sizeof desc->identifier - 1);
        }
        return CUT_OK;
    } catch (const Fail& f) {
        if (map != MAP_FAILED) ::munmap(map, map_bytes);
        if (fd >= 0) ::close(fd);
        return f.st;
    } catch (const std::bad_alloc&) {
        if (map != MAP_FAILED) ::munmap(map, map_bytes);
        if (fd >= 0) ::close(fd);
        set_error("cut_graph_build: out of host memory");
        return CUT_E_NOMEM;
    }
}

}  // namespace cut

using namespace cut;

extern "C" cut_status cut_graph_build(int32_t algebra, int32_t size, const char* path,
                                      int32_t threads, uint32_t flags, cut_graph_desc* desc) {
    int fd = -1;
    void* map = MAP_FAILED;
    size_t map_bytes = 0;
    try {
        auto t0 = std::chrono::steady_clock::now();
        if (!path) CUT_FAIL(CUT_E_INVAL, "cut_graph_build: null path");
        if (algebra == CUT_ALG_EPQ) {
            if (size < 1 || size > 64) CUT_FAIL(CUT_E_INVAL, "cut_graph_build: E_pq size %d outside 1..64", size);
        } else if (algebra == CUT_ALG_MAJORANA) {
            if (size < 4 || size > 64 || (size & 1))
                CUT_FAIL(CUT_E_INVAL, "cut_graph_build: Majorana size %d must be even in 4..64", size);
        } else if (algebra == CUT_ALG_PAULI_BOSON) {
            const int M = size / 256, pdeg = size % 256;
            if (M < 1 || M > 5 || pdeg < 1)
                CUT_FAIL(CUT_E_INVAL, "cut_graph_build: Pauli-boson size %d is not 256 M + p, M in 1..5, p >= 1", size);
            if (flags & ~CUT_BUILD_OUTSIDE) CUT_FAIL(CUT_E_INVAL, "cut_graph_build: unknown flags %#x", flags);
            const int nt = threads > 0 ? threads : (int)std::max(1u, std::thread::hardware_concurrency());
            return build_pauli_boson(M, pdeg, path, nt, (flags & CUT_BUILD_OUTSIDE) != 0, desc);
        } else {
            CUT_FAIL(CUT_E_INVAL, "cut_graph_build: unknown algebra %d", algebra);
        }
        if (flags & ~CUT_BUILD_OUTSIDE) CUT_FAIL(CUT_E_INVAL, "cut_graph_build: unknown flags %#x", flags);
        const bool outside = (flags & CUT_BUILD_OUTSIDE) != 0;
        if (outside && algebra != CUT_ALG_MAJORANA)
            CUT_FAIL(CUT_E_INVAL, "cut_graph_build: the E_pq registry is closed, it has no outside-space records");
        if (outside && size > 32)
            CUT_FAIL(CUT_E_UNSUPPORTED, "cut_graph_build: outside-space records only up to 32 modes");
        int nt = threads > 0 ? threads : (int)std::max(1u, std::thread::hardware_concurrency());
        Algebra alg(algebra, size);
        const int64_t N = alg.N;
        if (N >= (1ll << 31)) CUT_FAIL(CUT_E_UNSUPPORTED, "registry too large");

        // traversal 1: count records (and generator records) per target
        std::vector<int64_t> cntL(N + 1, 0), cntG(N + 1, 0);
        parallel_for(N, nt, [&](int64_t b, int64_t e) {
            std::vector<Rec> buf;
            for (int64_t k = b; k < e; ++k) {
                alg.expand(k, buf);
                int64_t g = 0;
                for (auto& r : buf) g += alg.diag[(size_t)r.i] ? 1 : 0;
                cntL[k + 1] = (int64_t)buf.size();
                cntG[k + 1] = g;
            }
        });
        for (int64_t k = 0; k < N; ++k) {
            cntL[k + 1] += cntL[k];
            cntG[k + 1] += cntG[k];
        }
        const int64_t E = cntL[N], Eg = cntG[N];
        // outside-space set E_C: same two traversals over the outside registry
        std::vector<uint64_t> olab;
        std::vector<int64_t> cntC(1, 0);
        if (outside) {
            olab = alg.outside_labels();
            cntC.assign(olab.size() + 1, 0);
            parallel_for((int64_t)olab.size(), nt, [&](int64_t b, int64_t e) {
                std::vector<Rec> buf;
                for (int64_t q = b; q < e; ++q) {
                    alg.expand_outside(olab[(size_t)q], buf);
                    cntC[q + 1] = (int64_t)buf.size();
                }
            });
            for (size_t q = 0; q < olab.size(); ++q) cntC[q + 1] += cntC[q];
        }
        const int64_t Nc = (int64_t)olab.size(), Ec = cntC.back();
        const int nsec = outside ? SEC_COUNT_OUT : SEC_COUNT;

        // exact section sizes -> file layout
        struct Sz {
            uint32_t id, eb;
            uint64_t count;
        } secs[SEC_COUNT_OUT] = {{SEC_LABELS, 8, (uint64_t)N},        {SEC_DIAG, 1, (uint64_t)N},
                                 {SEC_PAIRS, 4, alg.pairs.size()},     {SEC_FLOW_OFF, 8, (uint64_t)N + 1},
                                 {SEC_FLOW_I, 4, (uint64_t)E},         {SEC_FLOW_J, 4, (uint64_t)E},
                                 {SEC_FLOW_C, 1, (uint64_t)E},         {SEC_GEN_OFF, 8, (uint64_t)N + 1},
                                 {SEC_GEN_I, 4, (uint64_t)Eg},         {SEC_GEN_J, 4, (uint64_t)Eg},
                                 {SEC_GEN_C, 1, (uint64_t)Eg},         {SEC_OUT_LABELS, 8, (uint64_t)Nc},
                                 {SEC_OUT_OFF, 8, (uint64_t)Nc + 1},   {SEC_OUT_I, 4, (uint64_t)Ec},
                                 {SEC_OUT_J, 4, (uint64_t)Ec},         {SEC_OUT_C, 1, (uint64_t)Ec}};
        SectionEntry tab[SEC_COUNT_OUT];
        const size_t tab_bytes = nsec * sizeof(SectionEntry);
        uint64_t pos = align64(sizeof(BundleHeader) + tab_bytes);
        for (int s = 0; s < nsec; ++s) {
            tab[s] = {secs[s].id, secs[s].eb, pos, secs[s].count, 0};
            pos = align64(pos + secs[s].count * secs[s].eb);
        }
        const uint64_t file_bytes = pos;

        std::string tmp = std::string(path) + ".tmp";
        fd = ::open(tmp.c_str(), O_RDWR | O_CREAT | O_TRUNC, 0644);
        if (fd < 0) CUT_FAIL(CUT_E_IO, "cannot create %s", tmp.c_str());
        if (::ftruncate(fd, (off_t)file_bytes) != 0) CUT_FAIL(CUT_E_IO, "cannot size %s to %llu bytes", tmp.c_str(), (unsigned long long)file_bytes);
        map = ::mmap(nullptr, file_bytes, PROT_READ | PROT_WRITE, MAP_SHARED, fd, 0);
        if (map == MAP_FAILED) CUT_FAIL(CUT_E_IO, "cannot map %s", tmp.c_str());
        map_bytes = file_bytes;
        uint8_t* base = (uint8_t*)map;
        auto sec = [&](int s) { return base + tab[s].offset; };

        std::memcpy(sec(0), alg.labels.data(), N * 8);
        std::memcpy(sec(1), alg.diag.data(), N);
        std::memcpy(sec(2), alg.pairs.data(), alg.pairs.size() * 4);
        std::memcpy(sec(3), cntL.data(), (N + 1) * 8);
        std::memcpy(sec(7), cntG.data(), (N + 1) * 8);
        int32_t* Li = (int32_t*)sec(4);
        int32_t* Lj = (int32_t*)sec(5);
        int8_t* Lc = (int8_t*)sec(6);
        int32_t* Gi = (int32_t*)sec(8);
        int32_t* Gj = (int32_t*)sec(9);
        int8_t* Gc = (int8_t*)sec(10);
        if (outside) {
            std::memcpy(sec(11), olab.data(), Nc * 8);
            std::memcpy(sec(12), cntC.data(), (Nc + 1) * 8);
        }

        // traversal 2: regenerate and write every record in place
        parallel_for(N, nt, [&](int64_t b, int64_t e) {
            std::vector<Rec> buf;
            for (int64_t k = b; k < e; ++k) {
                alg.expand(k, buf);
                int64_t p = cntL[k], q = cntG[k];
                for (auto& r : buf) {
                    Li[p] = r.i;
                    Lj[p] = r.j;
                    Lc[p] = r.c;
                    ++p;
                    if (alg.diag[(size_t)r.i]) {
                        Gi[q] = r.i;
                        Gj[q] = r.j;
                        Gc[q] = r.c;
                        ++q;
                    }
                }
            }
        });

        if (outside) {
            int32_t* Ci = (int32_t*)sec(13);
            int32_t* Cj = (int32_t*)sec(14);
            int8_t* Cc = (int8_t*)sec(15);
            parallel_for(Nc, nt, [&](int64_t b, int64_t e) {
                std::vector<Rec> buf;
                for (int64_t q = b; q < e; ++q) {
                    alg.expand_outside(olab[(size_t)q], buf);
                    int64_t p = cntC[q];
                    for (auto& r : buf) {
                        Ci[p] = r.i;
                        Cj[p] = r.j;
                        Cc[p] = r.c;
                        ++p;
                    }
                }
            });
        }

        for (int s = 0; s < nsec; ++s) tab[s].checksum = checksum64(sec(s), tab[s].count * tab[s].elem_bytes);
        BundleHeader h{};
        std::memcpy(h.magic, kMagic, 8);
        h.version = kVersion;
        h.header_bytes = sizeof(BundleHeader);
        h.algebra = algebra;
        h.size = size;
        h.n_ops = N;
        h.n_records = E;
        h.n_gen_records = Eg;
        h.n_pairs = (int64_t)alg.pairs.size();
        h.factor_bytes = 1;
        h.gen_sign = alg.gen_sign;
        h.n_sections = (uint32_t)nsec;
        h.n_out_ops = Nc;
        h.n_out_records = Ec;
        h.section_table_offset = sizeof(BundleHeader);
        h.file_bytes = file_bytes;
        uint64_t rc = 0;
        for (int s = 3; s < nsec; ++s) rc = mix64(rc ^ tab[s].checksum);
        h.records_checksum = rc;
        std::string id = alg.identifier();
        std::strncpy(h.identifier, id.c_str(), sizeof h.identifier - 1);
        h.header_checksum = 0;
        std::memcpy(base + sizeof(BundleHeader), tab, tab_bytes);
        h.header_checksum = checksum64(&h, sizeof h) ^ checksum64(tab, tab_bytes);
        std::memcpy(base, &h, sizeof h);
        if (::msync(map, map_bytes, MS_SYNC) != 0) CUT_FAIL(CUT_E_IO, "msync failed");
        ::munmap(map, map_bytes);
        map = MAP_FAILED;
        ::close(fd);
        fd = -1;
        if (::rename(tmp.c_str(), path) != 0) CUT_FAIL(CUT_E_IO, "cannot rename %s to %s", tmp.c_str(), path);
        if (desc) {
            std::memset(desc, 0, sizeof *desc);
            desc->algebra = algebra;
            desc->size = size;
            desc->n_ops = N;
            desc->n_records = E;
            desc->n_gen_records = Eg;
            desc->n_pairs = h.n_pairs;
            desc->n_out_ops = Nc;
            desc->n_out_records = Ec;
            desc->checksum = rc;
            desc->file_bytes = (int64_t)file_bytes;
            desc->build_seconds =
                std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            std::strncpy(desc->identifier, h.identifier, sizeof desc->identifier - 1);
        }
        return CUT_OK;
    } catch (const Fail& f) {
        if (map != MAP_FAILED) ::munmap(map, map_bytes);
        if (fd >= 0) ::close(fd);
        return f.st;
    } catch (const std::bad_alloc&) {
        if (map != MAP_FAILED) ::munmap(map, map_bytes);
        if (fd >= 0) ::close(fd);
        set_error("cut_graph_build: out of host memory");
        return CUT_E_NOMEM;
    }
}

// ---------------------------------------------------------------- reader ----
namespace cut {

HostGraph::~HostGraph() {
    if (map) ::munmap(map, map_bytes);
}

void read_bundle(const char* path, bool verify, HostGraph& g) {
    int fd = ::open(path, O_RDONLY);
    if (fd < 0) CUT_FAIL(CUT_E_IO, "cannot open %s", path);
    struct stat st;
    if (::fstat(fd, &st) != 0) {
        ::close(fd);
        CUT_FAIL(CUT_E_IO, "cannot stat %s", path);
    }
    const uint64_t fbytes = (uint64_t)st.st_size;
    if (fbytes < sizeof(BundleHeader) + SEC_COUNT * sizeof(SectionEntry)) {
        ::close(fd);
        CUT_FAIL(CUT_E_FORMAT, "%s: truncated (%llu bytes)", path, (unsigned long long)fbytes);
    }
    void* map = ::mmap(nullptr, fbytes, PROT_READ, MAP_PRIVATE, fd, 0);
    ::close(fd);
    if (map == MAP_FAILED) CUT_FAIL(CUT_E_IO, "cannot map %s", path);
    g.map = map;
    g.map_bytes = fbytes;
    const uint8_t* base = (const uint8_t*)map;
    BundleHeader h;
    std::memcpy(&h, base, sizeof h);
    if (std::memcmp(h.magic, kMagic, 8) != 0) CUT_FAIL(CUT_E_FORMAT, "%s: not a graph bundle", path);
    if (h.version != kVersion || h.header_bytes != sizeof(BundleHeader))
        CUT_FAIL(CUT_E_FORMAT, "%s: unsupported bundle version %u", path, h.version);
    if (h.n_sections < (uint32_t)SEC_COUNT || h.n_sections > (uint32_t)kMaxSections ||
        h.section_table_offset != sizeof(BundleHeader))
        CUT_FAIL(CUT_E_FORMAT, "%s: bad section table", path);
    const int nsec = (int)h.n_sections;
    const size_t tab_bytes = nsec * sizeof(SectionEntry);
    if (fbytes < sizeof(BundleHeader) + tab_bytes) CUT_FAIL(CUT_E_FORMAT, "%s: truncated section table", path);
    if (h.file_bytes != fbytes) CUT_FAIL(CUT_E_FORMAT, "%s: size %llu, header says %llu", path,
                                         (unsigned long long)fbytes, (unsigned long long)h.file_bytes);
    SectionEntry tab[kMaxSections];
    std::memcpy(tab, base + sizeof h, tab_bytes);
    {
        BundleHeader hz = h;
        hz.header_checksum = 0;
        if ((checksum64(&hz, sizeof hz) ^ checksum64(tab, tab_bytes)) != h.header_checksum)
            CUT_FAIL(CUT_E_CHECKSUM, "%s: header checksum mismatch", path);
    }
    const int64_t N = h.n_ops;
    if (N <= 0 || h.n_records < 0 || h.n_gen_records < 0 || h.n_pairs < 0 || h.n_pairs > N || h.n_gen_ops < 0)
        CUT_FAIL(CUT_E_FORMAT, "%s: bad sizes", path);
    if ((h.factor_bytes != 1 && h.factor_bytes != 4 && h.factor_bytes != 16) || (h.gen_sign != 1 && h.gen_sign != -1))
        CUT_FAIL(CUT_E_FORMAT, "%s: bad factor format", path);
    const bool own_gen = h.n_gen_ops > 0;
    const int64_t NG = own_gen ? h.n_gen_ops : N;
    // expected section list: the base sections, the generator labels when the
    // generator has a registry of its own, then the outside-space sections
    struct Want {
        uint32_t id, eb;
        uint64_t count;
    };
    const uint32_t fb = (uint32_t)h.factor_bytes;
    std::vector<Want> want = {{SEC_LABELS, 8, (uint64_t)N},           {SEC_DIAG, 1, (uint64_t)N},
                              {SEC_PAIRS, 4, (uint64_t)h.n_pairs},     {SEC_FLOW_OFF, 8, (uint64_t)N + 1},
                              {SEC_FLOW_I, 4, (uint64_t)h.n_records},  {SEC_FLOW_J, 4, (uint64_t)h.n_records},
                              {SEC_FLOW_C, fb, (uint64_t)h.n_records}, {SEC_GEN_OFF, 8, (uint64_t)NG + 1},
                              {SEC_GEN_I, 4, (uint64_t)h.n_gen_records}, {SEC_GEN_J, 4, (uint64_t)h.n_gen_records},
                              {SEC_GEN_C, fb, (uint64_t)h.n_gen_records}};
    if (own_gen) want.push_back({SEC_GEN_LABELS, 8, (uint64_t)NG});
    const int out_at = (int)want.size();
    const bool outside = nsec == out_at + 5;
    if (!outside && nsec != out_at) CUT_FAIL(CUT_E_FORMAT, "%s: bad section count", path);
    if (outside ? (h.n_out_ops < 0 || h.n_out_records < 0) : (h.n_out_ops != 0 || h.n_out_records != 0))
        CUT_FAIL(CUT_E_FORMAT, "%s: bad outside-space sizes", path);
    if (outside) {
        want.push_back({SEC_OUT_LABELS, 8, (uint64_t)h.n_out_ops});
        want.push_back({SEC_OUT_OFF, 8, (uint64_t)h.n_out_ops + 1});
        want.push_back({SEC_OUT_I, 4, (uint64_t)h.n_out_records});
        want.push_back({SEC_OUT_J, 4, (uint64_t)h.n_out_records});
        want.push_back({SEC_OUT_C, fb, (uint64_t)h.n_out_records});
    }
    const void* ptr[kMaxSections];
    for (int s = 0; s < nsec; ++s) {
        const SectionEntry& e = tab[s];
        if (e.id != want[s].id || e.count != want[s].count || e.elem_bytes != want[s].eb || (e.offset & 63) ||
            e.offset < sizeof h + tab_bytes || e.offset > fbytes || e.count * e.elem_bytes > fbytes - e.offset)
            CUT_FAIL(CUT_E_FORMAT, "%s: section %d malformed", path, s);
        ptr[s] = base + e.offset;
    }
    if (verify) {
        for (int s = 0; s < nsec; ++s)
            if (checksum64(ptr[s], tab[s].count * tab[s].elem_bytes) != tab[s].checksum)
                CUT_FAIL(CUT_E_CHECKSUM, "%s: section %d checksum mismatch", path, s);
    }
    g.hdr = h;
    g.n_gen = NG;
    g.labels = (const uint64_t*)ptr[0];
    g.diag = (const uint8_t*)ptr[1];
    g.pairs = (const int32_t*)ptr[2];
    for (int w = 0; w < 2; ++w) {
        g.off[w] = (const int64_t*)ptr[3 + 4 * w];
        g.ri[w] = (const int32_t*)ptr[4 + 4 * w];
        g.rj[w] = (const int32_t*)ptr[5 + 4 * w];
        g.rc[w] = (const int8_t*)ptr[6 + 4 * w];
    }
    if (own_gen) g.gen_labels = (const uint64_t*)ptr[11];
    if (outside) {
        g.out_labels = (const uint64_t*)ptr[out_at];
        g.off[2] = (const int64_t*)ptr[out_at + 1];
        g.ri[2] = (const int32_t*)ptr[out_at + 2];
        g.rj[2] = (const int32_t*)ptr[out_at + 3];
        g.rc[2] = (const int8_t*)ptr[out_at + 4];
    }
    // structural validation: offsets monotone and complete, indices in range
    // (left inputs of E_L and E_C are generator rows, everything else operator
    // rows), factors nonzero and finite
    for (int w = 0; w < (outside ? 3 : 2); ++w) {
        const int64_t E = w == 0 ? h.n_records : w == 1 ? h.n_gen_records : h.n_out_records;
        const int64_t nseg = w == 2 ? h.n_out_ops : w == 1 ? NG : N;
        const uint64_t ilim = (uint64_t)(w == 1 ? N : NG);
        const int64_t* off = g.off[w];
        if (off[0] != 0 || off[nseg] != E) CUT_FAIL(CUT_E_FORMAT, "%s: offsets incomplete", path);
        for (int64_t k = 0; k < nseg; ++k)
            if (off[k + 1] < off[k]) CUT_FAIL(CUT_E_FORMAT, "%s: offsets not monotone at %lld", path, (long long)k);
        const int32_t* ri = g.ri[w];
        const int32_t* rj = g.rj[w];
        const int8_t* rc = g.rc[w];
        std::atomic<int> bad{0};
        parallel_for(E, 16, [&](int64_t b, int64_t e) {
            for (int64_t t = b; t < e; ++t) {
                bool zero;
                if (fb == 1) {
                    zero = rc[t] == 0;
                } else if (fb == 4) {
                    int16_t re, im;
                    std::memcpy(&re, rc + 4 * t, 2);
                    std::memcpy(&im, rc + 4 * t + 2, 2);
                    zero = re == 0 && im == 0;
                } else {
                    double re, im;
                    std::memcpy(&re, rc + 16 * t, 8);
                    std::memcpy(&im, rc + 16 * t + 8, 8);
                    zero = (re == 0 && im == 0) || !std::isfinite(re) || !std::isfinite(im);
                }
                if ((uint32_t)ri[t] >= ilim || (uint32_t)rj[t] >= (uint64_t)N || zero) bad = 1;
            }
        });
        if (bad) CUT_FAIL(CUT_E_FORMAT, "%s: record index out of range or zero factor", path);
    }
    for (int64_t t = 0; t < h.n_pairs; ++t)
        if ((uint32_t)g.pairs[t] >= (uint64_t)N) CUT_FAIL(CUT_E_FORMAT, "%s: pair index out of range", path);
}

}  // namespace cut
