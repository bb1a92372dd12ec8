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
#include <cstring>
#include <functional>
#include <thread>

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
    if ((h.n_sections != SEC_COUNT && h.n_sections != SEC_COUNT_OUT) ||
        h.section_table_offset != sizeof(BundleHeader))
        CUT_FAIL(CUT_E_FORMAT, "%s: bad section table", path);
    const int nsec = (int)h.n_sections;
    const size_t tab_bytes = nsec * sizeof(SectionEntry);
    if (fbytes < sizeof(BundleHeader) + tab_bytes) CUT_FAIL(CUT_E_FORMAT, "%s: truncated section table", path);
    if (h.file_bytes != fbytes) CUT_FAIL(CUT_E_FORMAT, "%s: size %llu, header says %llu", path,
                                         (unsigned long long)fbytes, (unsigned long long)h.file_bytes);
    SectionEntry tab[SEC_COUNT_OUT];
    std::memcpy(tab, base + sizeof h, tab_bytes);
    {
        BundleHeader hz = h;
        hz.header_checksum = 0;
        if ((checksum64(&hz, sizeof hz) ^ checksum64(tab, tab_bytes)) != h.header_checksum)
            CUT_FAIL(CUT_E_CHECKSUM, "%s: header checksum mismatch", path);
    }
    const int64_t N = h.n_ops;
    if (N <= 0 || h.n_records < 0 || h.n_gen_records < 0 || h.n_pairs < 0 || h.n_pairs > N)
        CUT_FAIL(CUT_E_FORMAT, "%s: bad sizes", path);
    const bool outside = nsec == SEC_COUNT_OUT;
    if (outside ? (h.n_out_ops < 0 || h.n_out_records < 0) : (h.n_out_ops != 0 || h.n_out_records != 0))
        CUT_FAIL(CUT_E_FORMAT, "%s: bad outside-space sizes", path);
    if (h.factor_bytes != 1 || (h.gen_sign != 1 && h.gen_sign != -1))
        CUT_FAIL(CUT_E_FORMAT, "%s: bad factor format", path);
    const uint64_t want[SEC_COUNT_OUT][2] = {
        {SEC_LABELS, (uint64_t)N},          {SEC_DIAG, (uint64_t)N},
        {SEC_PAIRS, (uint64_t)h.n_pairs},   {SEC_FLOW_OFF, (uint64_t)N + 1},
        {SEC_FLOW_I, (uint64_t)h.n_records}, {SEC_FLOW_J, (uint64_t)h.n_records},
        {SEC_FLOW_C, (uint64_t)h.n_records}, {SEC_GEN_OFF, (uint64_t)N + 1},
        {SEC_GEN_I, (uint64_t)h.n_gen_records}, {SEC_GEN_J, (uint64_t)h.n_gen_records},
        {SEC_GEN_C, (uint64_t)h.n_gen_records}, {SEC_OUT_LABELS, (uint64_t)h.n_out_ops},
        {SEC_OUT_OFF, (uint64_t)h.n_out_ops + 1}, {SEC_OUT_I, (uint64_t)h.n_out_records},
        {SEC_OUT_J, (uint64_t)h.n_out_records}, {SEC_OUT_C, (uint64_t)h.n_out_records}};
    const uint32_t eb[SEC_COUNT_OUT] = {8, 1, 4, 8, 4, 4, 1, 8, 4, 4, 1, 8, 8, 4, 4, 1};
    const void* ptr[SEC_COUNT_OUT];
    for (int s = 0; s < nsec; ++s) {
        const SectionEntry& e = tab[s];
        if (e.id != want[s][0] || e.count != want[s][1] || e.elem_bytes != eb[s] || (e.offset & 63) ||
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
    g.labels = (const uint64_t*)ptr[0];
    g.diag = (const uint8_t*)ptr[1];
    g.pairs = (const int32_t*)ptr[2];
    for (int w = 0; w < 2; ++w) {
        g.off[w] = (const int64_t*)ptr[3 + 4 * w];
        g.ri[w] = (const int32_t*)ptr[4 + 4 * w];
        g.rj[w] = (const int32_t*)ptr[5 + 4 * w];
        g.rc[w] = (const int8_t*)ptr[6 + 4 * w];
    }
    if (outside) {
        g.out_labels = (const uint64_t*)ptr[11];
        g.off[2] = (const int64_t*)ptr[12];
        g.ri[2] = (const int32_t*)ptr[13];
        g.rj[2] = (const int32_t*)ptr[14];
        g.rc[2] = (const int8_t*)ptr[15];
    }
    // structural validation: offsets monotone and complete, indices in range
    for (int w = 0; w < (outside ? 3 : 2); ++w) {
        const int64_t E = w == 0 ? h.n_records : w == 1 ? h.n_gen_records : h.n_out_records;
        const int64_t nseg = w == 2 ? h.n_out_ops : N;
        const int64_t* off = g.off[w];
        if (off[0] != 0 || off[nseg] != E) CUT_FAIL(CUT_E_FORMAT, "%s: offsets incomplete", path);
        for (int64_t k = 0; k < nseg; ++k)
            if (off[k + 1] < off[k]) CUT_FAIL(CUT_E_FORMAT, "%s: offsets not monotone at %lld", path, (long long)k);
        const int32_t* ri = g.ri[w];
        const int32_t* rj = g.rj[w];
        const int8_t* rc = g.rc[w];
        std::atomic<int> bad{0};
        parallel_for(E, 16, [&](int64_t b, int64_t e) {
            for (int64_t t = b; t < e; ++t)
                if ((uint32_t)ri[t] >= (uint64_t)N || (uint32_t)rj[t] >= (uint64_t)N || rc[t] == 0) bad = 1;
        });
        if (bad) CUT_FAIL(CUT_E_FORMAT, "%s: record index out of range or zero factor", path);
    }
    for (int64_t t = 0; t < h.n_pairs; ++t)
        if ((uint32_t)g.pairs[t] >= (uint64_t)N) CUT_FAIL(CUT_E_FORMAT, "%s: pair index out of range", path);
}

}  // namespace cut
