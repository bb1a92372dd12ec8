// Graph load: validated reload of a bundle (Sec. 2.3) and the device layout.
//
// Device layout per record set (E_L, E_eta):
//   orientation 0: grouped by target k, records (a=i, b=j); Majorana graphs in
//   locality order (by shared triple), others in stored (i, j) order
//   orientation 1: grouped by right input j, records (a=i, b=k), ordered (k, i)
//   orientation 2: grouped by left input i, records (a=k, b=j), ordered (k, j)
// Orientations 1 and 2 are the reverse traversals of the same records used by
// the adjoint (Sec. 2.4); they are built by a stable counting sort on the host.
// Each record is 8 bytes: uint32 (f_hi << 24 | a), uint32 (f_lo << 24 | b), where
// (f_hi, f_lo) is the bf16 bit pattern of the integer factor (exact for int8).
#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <unordered_map>

#include "internal.h"

namespace cut {

static thread_local char g_err[512] = "";

void set_error(const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

template <class T>
static T* dev_alloc(size_t n) {
    void* p = nullptr;
    if (n == 0) n = 1;
    hipError_t e = hipMalloc(&p, n * sizeof(T));
    if (e != hipSuccess) CUT_FAIL(CUT_E_NOMEM, "hipMalloc(%zu bytes): %s", n * sizeof(T), hipGetErrorString(e));
    return (T*)p;
}

template <class T>
static void dev_free(T*& p) {
    if (p) (void)hipFree((void*)p);
    p = nullptr;
}

void ChunkPlan::release() {
    dev_free(short_tasks);
    dev_free(chunks);
    dev_free(cstart);
    dev_free(crow);
    nshort = short_per_xcd = nchunks = nlong = nslots = 0;
}

void QuadBlockPlan::release_tiling() {
    dev_free(tslot);
    cp.release();
    cp_lead.release();
    active = false;
}

void QuadBlockPlan::release() {
    release_tiling();
    dev_free(row4);
    dev_free(tmask);
    dev_free(bpair);
    dev_free(sgn);
    fmag = 0.f;
    qrow.clear();
    lead.clear();
    ok = false;
    m = ng = nbp = nr = 0;
    ntrip = 0;
}

void DevCSR::release() {
    dev_free(off);
    dev_free(rec);
    dev_free(tasks);
    cp.release();
    off_h.clear();
    off_h.shrink_to_fit();
    nseg = nrec = ntasks = per_xcd = 0;
}

void* Workspace::need(size_t n, const char* what) const {
    if (n <= bytes) return ptr;
    CUT_FAIL(CUT_E_INVAL,
             "%s needs a work area of %zu bytes, %zu are reserved: call cut_graph_reserve with this shape "
             "(and again after a tiling change that adds partial rows)",
             what, n, bytes);
}

void Workspace::reserve(size_t n) {
    if (n <= bytes) return;
    if (ptr) {
        HIP_CHECK(hipDeviceSynchronize());
        (void)hipFree(ptr);
        ptr = nullptr;
        bytes = 0;
    }
    hipError_t e = hipMalloc(&ptr, n);
    if (e != hipSuccess) {
        ptr = nullptr;
        CUT_FAIL(CUT_E_NOMEM, "work area hipMalloc(%zu): %s", n, hipGetErrorString(e));
    }
    bytes = n;
}

void Workspace::release() {
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

void release_step_graphs(Graph& g);

Graph::~Graph() {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(device);
    release_step_graphs(*this);
    for (auto& w : csr)
        for (auto& c : w) c.release();
    for (auto& c : cxs) c.release();
    dev_free(ftab);
    dev_free(diag);
    dev_free(pairs);
    dev_free(stencil);
    dev_free(st_t_off);
    dev_free(st_t);
    dev_free(st_p_off);
    dev_free(st_p);
    tiles.release();
    qb.release();
    ws.release();
    ws_small.release();
    ws_part.release();
    ws_deriv.release();
    (void)hipSetDevice(cur);
}

// Tiling plan.  Targets longer than long_records become one task split over the
// four wavefronts; shorter consecutive targets are packed four per task.  With
// XCD remapping, the target range is cut into 8 contiguous pieces of equal
// record count (one per XCD, so neighbouring targets share one L2), each piece
// lists its long tasks first; shorter lists are padded with empty tasks.
static std::vector<Task> plan_tasks(const Graph& g, const std::vector<int64_t>& off, int64_t nseg, int64_t* per_xcd);

static void upload_tasks(const std::vector<Task>& all, Task** dst, int64_t* n) {
    dev_free(*dst);
    *n = (int64_t)all.size();
    if (all.empty()) return;
    *dst = dev_alloc<Task>(all.size());
    HIP_CHECK(hipMemcpy(*dst, all.data(), all.size() * sizeof(Task), hipMemcpyHostToDevice));
}

// Lexicographic rank of a 3-subset {a < b < c} of [0, m) (hockey-stick form).
static int64_t lex_rank3(uint64_t t, int m) {
    auto c3 = [](int64_t a) { return a < 3 ? 0 : a * (a - 1) * (a - 2) / 6; };
    auto c2 = [](int64_t a) { return a < 2 ? 0 : a * (a - 1) / 2; };
    int e[3], r = 0;
    for (uint64_t x = t; x && r < 3; x &= x - 1) e[r++] = __builtin_ctzll(x);
    return (c3(m) - c3(m - e[0])) + (c2(m - e[0] - 1) - c2(m - e[1])) + ((m - e[1] - 1) - (m - e[2]));
}

// Chunked plan.  Every segment longer than long_records is cut into
// ceil(len / chunk_records) near-equal chunks, placed at the relative position
// of their midpoint in the segment (chunks at the same position of different
// long segments read the same operand rows once the segments are in locality
// order).  With triple chunks (Majorana graphs whose quartic targets come in 4
// shared-triple groups), every quartic target is cut into chunks of whole
// groups, about chunk_records records each, placed at the rank of the chunk's
// first triple among all triples; the chunks of the targets that share a triple
// then run together and read that triple's rows.  Chunks are listed by
// position; partial-row slots are numbered per segment in chunk order.  With
// XCD remapping the list is cut into 8 contiguous pieces, piece x running on
// XCD x (block b on XCD b % 8), padded with empty chunks.  The remaining short
// segments are packed four per task (same XCD split).
// With `quad` (quadratic-target blocks) every quadratic target becomes one
// chunk of its leading records followed by qb.nr partial slots that the block
// kernel fills; seg_slot[k] receives the first of those block slots.
static void build_chunks(const Graph& g, const DevCSR& c, ChunkPlan& out, bool quad,
                         std::vector<int64_t>* seg_slot = nullptr, bool skip_quartic = false) {
    out.release();
    const std::vector<int64_t>& off = c.off_h;
    const int64_t lr = g.long_records, cr = std::max<int64_t>(1, g.chunk_records);
    std::vector<int64_t> cstart = {0};
    std::vector<int32_t> crow;
    struct Ent {
        double pos;
        ChunkTask t;
    };
    std::vector<Ent> ents;
    std::vector<uint8_t> is_long(c.nseg, 0);
    if (c.nrec >= (1ll << 31) || !g.use_chunks) return;
    const int m = g.hdr.size;
    const bool fam = g.triple_chunks && g.triple_groups && g.hdr.algebra == CUT_ALG_MAJORANA &&
                     (int64_t)g.labels_h.size() == c.nseg && m >= 4;
    const double ntrip = (double)m * (m - 1) * (m - 2) / 6.0;
    if (seg_slot) seg_slot->assign(c.nseg, -1);
    for (int64_t k = 0; k < c.nseg; ++k) {
        const int64_t len = off[k + 1] - off[k];
        if (skip_quartic && __builtin_popcountll(g.labels_h[k]) == 4) {
            is_long[k] = 1;  // handled by the tile kernel: neither chunk nor short task
            continue;
        }
        const bool quart = fam && len > 0 && __builtin_popcountll(g.labels_h[k]) == 4;
        const bool qtarget = quad && __builtin_popcountll(g.labels_h[k]) == 2;
        if (!quart && !qtarget && len <= lr) continue;
        is_long[k] = 1;
        const int64_t l = (int64_t)crow.size();
        crow.push_back((int32_t)k);
        int64_t nch = 0;
        if (qtarget) {
            // leading records in one chunk (slot 0), then the block slots
            ents.push_back({0.0, ChunkTask{(int32_t)k, (int32_t)cstart[l], (int32_t)off[k],
                                           (int32_t)(off[k] + g.qb.lead[k])}});
            if (seg_slot) (*seg_slot)[k] = cstart[l] + 1;
            nch = 1 + g.qb.nr;
        } else if (quart) {
            const int64_t q = len / 4;
            const int gpc = (int)std::min<int64_t>(4, std::max<int64_t>(1, (cr + q / 2) / q));
            int e[4], r = 0;
            for (uint64_t x = g.labels_h[k]; x && r < 4; x &= x - 1) e[r++] = __builtin_ctzll(x);
            for (int t0 = 0; t0 < 4; t0 += gpc, ++nch) {
                const int t1 = std::min(4, t0 + gpc);
                // group t of K = {e0<e1<e2<e3} reads the rows of the triple K - e[3-t]
                const uint64_t T = g.labels_h[k] & ~(1ull << e[3 - t0]);
                ents.push_back({(double)lex_rank3(T, m) / ntrip,
                                ChunkTask{(int32_t)k, (int32_t)(cstart[l] + nch), (int32_t)(off[k] + t0 * q),
                                          (int32_t)(off[k] + t1 * q)}});
            }
        } else {
            nch = (len + cr - 1) / cr;
            for (int64_t q = 0; q < nch; ++q) {
                const int64_t e0 = off[k] + len * q / nch, e1 = off[k] + len * (q + 1) / nch;
                ents.push_back({(q + 0.5) / nch, ChunkTask{(int32_t)k, (int32_t)(cstart[l] + q), (int32_t)e0, (int32_t)e1}});
            }
        }
        cstart.push_back(cstart[l] + nch);
    }
    std::stable_sort(ents.begin(), ents.end(), [](const Ent& a, const Ent& b) { return a.pos < b.pos; });
    std::vector<ChunkTask> ch;
    const ChunkTask pad{-1, 0, 0, 0};
    if (g.xcd_remap && !ents.empty()) {
        const int64_t nblk = ((int64_t)ents.size() + 3) / 4, per = (nblk + 7) / 8;
        ch.assign((size_t)(8 * per * 4), pad);
        for (int64_t b = 0; b < 8 * per; ++b) {
            const int64_t src = (b % 8) * per + b / 8;  // block of the sorted list
            for (int w = 0; w < 4; ++w) {
                const int64_t i = src * 4 + w;
                if (src < nblk && i < (int64_t)ents.size()) ch[b * 4 + w] = ents[i].t;
            }
        }
    } else {
        ch.reserve(ents.size());
        for (auto& e : ents) ch.push_back(e.t);
    }
    // short segments: packed tasks over maximal runs of short segments
    auto pack = [&](int64_t b, int64_t e, std::vector<Task>& out) {
        for (int64_t k = b; k < e;) {
            if (is_long[k]) {
                ++k;
                continue;
            }
            int64_t k0 = k;
            int n = 0;
            while (k < e && n < 4 && !is_long[k]) {
                ++k;
                ++n;
            }
            out.push_back({(int32_t)k0, n});
        }
    };
    std::vector<Task> st;
    if (g.xcd_remap) {
        int64_t total = 0;
        for (int64_t k = 0; k < c.nseg; ++k)
            if (!is_long[k]) total += off[k + 1] - off[k] + 64;
        std::vector<std::vector<Task>> parts(8);
        int64_t b = 0, acc = 0;
        for (int x = 0; x < 8; ++x) {
            int64_t e = b;
            const int64_t goal = total * (x + 1) / 8;
            while (e < c.nseg && (x == 7 || acc < goal)) {
                if (!is_long[e]) acc += off[e + 1] - off[e] + 64;
                ++e;
            }
            pack(b, e, parts[x]);
            b = e;
        }
        size_t per = 0;
        for (auto& p : parts) per = std::max(per, p.size());
        if (per > 0) {
            st.assign(per * 8, Task{0, 0});
            for (int x = 0; x < 8; ++x) std::copy(parts[x].begin(), parts[x].end(), st.begin() + x * per);
            out.short_per_xcd = (int64_t)per;
        }
    } else {
        pack(0, c.nseg, st);
    }
    out.nshort = (int64_t)st.size();
    if (!st.empty()) {
        out.short_tasks = dev_alloc<Task>(st.size());
        HIP_CHECK(hipMemcpy(out.short_tasks, st.data(), st.size() * sizeof(Task), hipMemcpyHostToDevice));
    }
    out.nlong = (int64_t)crow.size();
    out.nchunks = (int64_t)ch.size();
    out.nslots = cstart.back();
    if (out.nlong == 0) return;
    if (!ch.empty()) {
        out.chunks = dev_alloc<ChunkTask>(ch.size());
        HIP_CHECK(hipMemcpy(out.chunks, ch.data(), ch.size() * sizeof(ChunkTask), hipMemcpyHostToDevice));
    }
    out.cstart = dev_alloc<int64_t>(cstart.size());
    HIP_CHECK(hipMemcpy(out.cstart, cstart.data(), cstart.size() * 8, hipMemcpyHostToDevice));
    out.crow = dev_alloc<int32_t>(crow.size());
    HIP_CHECK(hipMemcpy(out.crow, crow.data(), crow.size() * 4, hipMemcpyHostToDevice));
}

// Per-tiling tables of the quadratic-target blocks: the chunked form with the
// leading records of every quadratic target as chunks, and for every block
// pair and local target t = 8 iu + iv (u = 8 g1 + iu, v = 8 g2 + iv, u < v) its
// first block partial slot (range r of triples [r ntrip / nr, (r+1) ntrip / nr)
// in lexicographic order goes to slot + r).
static void build_qb_tiling(Graph& g, const DevCSR& c) {
    QuadBlockPlan& q = g.qb;
    q.release_tiling();
    if (!q.ok || !g.use_quadblocks || !g.use_chunks || c.nrec >= (1ll << 31)) return;
    std::vector<int64_t> seg_slot;
    build_chunks(g, c, q.cp, true, &seg_slot);
    if (g.use_tiles && g.tiles.ok) {
        // same slots for the quadratic targets: their rows precede the quartic ones
        std::vector<int64_t> seg_lead;
        build_chunks(g, c, q.cp_lead, true, &seg_lead, true);
        for (int64_t k = 0; k < c.nseg; ++k)
            if (__builtin_popcountll(g.labels_h[k]) == 2 && seg_lead[k] != seg_slot[k])
                CUT_FAIL(CUT_E_FORMAT, "quadratic-target blocks: slot numbering mismatch");
    }
    const int m = q.m;
    std::vector<int32_t> tslot((size_t)q.nbp * 64, -1);
    int bp = 0;
    for (int g1 = 0; g1 < q.ng; ++g1)
        for (int g2 = g1; g2 < q.ng; ++g2, ++bp)
            for (int t = 0; t < 64; ++t) {
                const int u = 8 * g1 + t / 8, v = 8 * g2 + t % 8;
                if (u >= m || v >= m || u >= v) continue;
                tslot[(size_t)bp * 64 + t] = (int32_t)seg_slot[q.qrow[u * m + v]];
            }
    q.tslot = dev_alloc<int32_t>(tslot.size());
    HIP_CHECK(hipMemcpy(q.tslot, tslot.data(), tslot.size() * 4, hipMemcpyHostToDevice));
    q.active = true;
}

void build_tasks(Graph& g, DevCSR& c) {
    ++g.tiling_gen;
    c.per_xcd = 0;
    if (c.nseg == 0) {
        upload_tasks({}, &c.tasks, &c.ntasks);
        return;
    }
    upload_tasks(plan_tasks(g, c.off_h, c.nseg, &c.per_xcd), &c.tasks, &c.ntasks);
    if (&c == &g.csr[0][0]) {
        build_chunks(g, c, c.cp, false);
        build_qb_tiling(g, c);
    }
    if (&c == &g.csr[0][0] && g.tiles.ok) {
        g.tiles.res_per_xcd = 0;
        upload_tasks(plan_tasks(g, c.off_h, g.tiles.nres, &g.tiles.res_per_xcd), &g.tiles.res_tasks,
                     &g.tiles.nres_tasks);
    }
}

void apply_tiling(Graph& g, int64_t long_records, int64_t chunk_records, uint32_t flags) {
    g.long_records = long_records;
    g.chunk_records = chunk_records;
    g.xcd_remap = (flags & CUT_TILE_XCD_REMAP) ? 1 : 0;
    g.use_tiles = (flags & CUT_TILE_TRIPLES) ? 1 : 0;
    g.use_chunks = (flags & CUT_TILE_NO_CHUNKS) ? 0 : 1;
    g.triple_chunks = (flags & CUT_TILE_TRIPLE_CHUNKS) ? 1 : 0;
    g.use_quadblocks = (flags & CUT_TILE_QUAD_BLOCKS) ? 1 : 0;
    g.bchunk = (int)((flags >> CUT_TILE_BCHUNK_SHIFT) & 3u);
    for (auto& w : g.csr)
        for (auto& c : w)
            if (c.nseg) build_tasks(g, c);
}

uint32_t tiling_flags(const Graph& g) {
    return (g.xcd_remap ? CUT_TILE_XCD_REMAP : 0u) | (g.use_tiles ? CUT_TILE_TRIPLES : 0u) |
           (g.use_chunks ? 0u : CUT_TILE_NO_CHUNKS) | (g.triple_chunks ? CUT_TILE_TRIPLE_CHUNKS : 0u) |
           (g.use_quadblocks ? CUT_TILE_QUAD_BLOCKS : 0u) | ((uint32_t)g.bchunk << CUT_TILE_BCHUNK_SHIFT);
}

static std::vector<Task> plan_tasks(const Graph& g, const std::vector<int64_t>& off, int64_t nseg, int64_t* per_xcd) {
    auto plan = [&](int64_t b, int64_t e, std::vector<Task>& out) {
        std::vector<Task> shorts;
        for (int64_t k = b; k < e;) {
            if (off[k + 1] - off[k] > g.long_records) {
                out.push_back({(int32_t)k, -1});
                ++k;
                continue;
            }
            int64_t k0 = k;
            int n = 0;
            while (k < e && n < 4 && off[k + 1] - off[k] <= g.long_records) {
                ++k;
                ++n;
            }
            shorts.push_back({(int32_t)k0, n});
        }
        out.insert(out.end(), shorts.begin(), shorts.end());
    };
    std::vector<Task> all;
    *per_xcd = 0;
    if (nseg == 0) return all;
    if (g.xcd_remap) {
        std::vector<std::vector<Task>> parts(8);
        const int64_t total = off[nseg] + 64 * nseg;  // records + per-target overhead
        int64_t b = 0;
        for (int x = 0; x < 8; ++x) {
            int64_t e = b;
            const int64_t goal = total * (x + 1) / 8;
            while (e < nseg && (off[e] + 64 * e) < goal) ++e;
            if (x == 7) e = nseg;
            plan(b, e, parts[x]);
            b = e;
        }
        size_t per = 0;
        for (auto& p : parts) per = std::max(per, p.size());
        all.assign(per * 8, Task{0, 0});
        for (int x = 0; x < 8; ++x) std::copy(parts[x].begin(), parts[x].end(), all.begin() + x * per);
        *per_xcd = (int64_t)per;
    } else {
        plan(0, nseg, all);
    }
    return all;
}

void TilePlan::release() {
    dev_free(rows);
    dev_free(slot);
    dev_free(rec);
    dev_free(res_tasks);
    ntiles = nres_tasks = res_per_xcd = nres = 0;
    ok = false;
}

// Shared-triple tile plan for Majorana registries, derived from the registry
// labels and the E_L records: for every record of a quartic target K whose
// other operands are a quadratic string and a quartic K' with |K & K'| = 3,
// tau = K & K' names the tile, w = K \ tau the member and q = K' \ tau the
// staged operand (local index = mode minus the tau modes below it).  The plan is
// accepted only if every quartic-target record lands in exactly one tile slot
// and every (tile, member) holds the same number of records.
static void build_tiles(Graph& g, const HostGraph& hg, const uint8_t* code) {
    if (hg.hdr.algebra != CUT_ALG_MAJORANA) return;
    const int m = hg.hdr.size;
    const int64_t N = hg.hdr.n_ops;
    const int64_t nquad = (int64_t)m * (m - 1) / 2;
    const int M = m - 3, RT = 2 * (m - 4);
    if (M < 2 || RT < 1) return;
    auto binom3 = [](int64_t a) { return a < 3 ? 0 : a * (a - 1) * (a - 2) / 6; };
    const int64_t ntiles = binom3(m);
    // lexicographic rank of a 3-subset {a < b < c} of [0, m)
    std::vector<int64_t> c3(m + 1), c2(m + 1);
    for (int a = 0; a <= m; ++a) {
        c3[a] = binom3(a);
        c2[a] = (int64_t)a * (a - 1) / 2;
    }
    auto rank3 = [&](uint64_t t) {
        int e[3], r = 0;
        for (uint64_t x = t; x; x &= x - 1) e[r++] = __builtin_ctzll(x);
        // hockey-stick form of the lexicographic rank
        return (c3[m] - c3[m - e[0]]) + (c2[m - e[0] - 1] - c2[m - e[1]]) + ((m - e[1] - 1) - (m - e[2]));
    };
    auto local = [](uint64_t tau, int mode) { return mode - __builtin_popcountll(tau & ((1ull << mode) - 1)); };
    const int64_t* off = hg.off[0];
    for (int64_t k = nquad; k < N; ++k)
        if (off[k + 1] - off[k] != 4 * (int64_t)RT) return;
    std::vector<int32_t> rows(ntiles * M, -1);
    std::vector<uint8_t> slot(ntiles * M, 255);
    std::vector<uint2> rec(ntiles * M * (size_t)RT);
    std::vector<int32_t> fill(ntiles * M, 0);
    for (int64_t k = nquad; k < N; ++k) {
        const uint64_t K = hg.labels[k];
        if (__builtin_popcountll(K) != 4) return;
        for (int64_t e = off[k]; e < off[k + 1]; ++e) {
            const int32_t i = hg.ri[0][e], j = hg.rj[0][e];
            const uint64_t Li = hg.labels[i], Lj = hg.labels[j];
            const int orient = __builtin_popcountll(Li) == 4 ? 1 : 0;  // 1: generator row is quartic
            const uint64_t Q = orient ? Li : Lj;
            const int32_t quad = orient ? j : i;
            if (__builtin_popcountll(hg.labels[quad]) != 2 || __builtin_popcountll(Q) != 4) return;
            const uint64_t tau = K & Q;
            if (__builtin_popcountll(tau) != 3) return;
            const int w = __builtin_ctzll(K & ~tau), q = __builtin_ctzll(Q & ~tau);
            const int64_t tile = rank3(tau);
            if (tile < 0 || tile >= ntiles) return;
            const int64_t mt = tile * M + local(tau, w);
            const int sl = __builtin_popcountll(K & ((1ull << w) - 1));
            if (rows[mt] < 0) {
                rows[mt] = (int32_t)k;
                slot[mt] = (uint8_t)sl;
            } else if (rows[mt] != k || slot[mt] != sl) {
                return;
            }
            if (fill[mt] >= RT) return;
            // factor as the top half of its FP32 bit pattern (exact for int8)
            const float f = (float)hg.rc[0][e];
            uint32_t fb;
            std::memcpy(&fb, &f, 4);
            rec[mt * RT + fill[mt]++] =
                make_uint2((uint32_t)quad, (fb & 0xFFFF0000u) | ((uint32_t)local(tau, q) << 1) | (uint32_t)orient);
        }
    }
    for (int64_t mt = 0; mt < ntiles * M; ++mt)
        if (fill[mt] != RT || rows[mt] < 0) return;
    // within each member: records whose generator is the quadratic row first
    // (operand from LDS), then the others, each in stored order; the two halves
    // must be equal (every partner T+q contributes one record of each kind)
    for (int64_t mt = 0; mt < ntiles * M; ++mt) {
        uint2* r = rec.data() + mt * RT;
        std::stable_sort(r, r + RT, [](const uint2& x, const uint2& y) { return (x.y & 1u) < (y.y & 1u); });
        if (RT % 2 != 0 || (r[RT / 2 - 1].y & 1u) != 0 || (r[RT / 2].y & 1u) != 1) return;
    }
    TilePlan& tp = g.tiles;
    tp.ntiles = ntiles;
    tp.M = M;
    tp.RT = RT;
    tp.nres = nquad;
    tp.rows = dev_alloc<int32_t>(rows.size());
    HIP_CHECK(hipMemcpy(tp.rows, rows.data(), rows.size() * 4, hipMemcpyHostToDevice));
    tp.slot = dev_alloc<uint8_t>(slot.size());
    HIP_CHECK(hipMemcpy(tp.slot, slot.data(), slot.size(), hipMemcpyHostToDevice));
    tp.rec = dev_alloc<uint2>(rec.size());
    HIP_CHECK(hipMemcpy(tp.rec, rec.data(), rec.size() * sizeof(uint2), hipMemcpyHostToDevice));
    tp.ok = true;
    build_tasks(g, g.csr[0][0]);
}

static void upload_csr(Graph& g, DevCSR& c, int64_t nseg, std::vector<int64_t>&& off,
                       const std::vector<uint2>& rec) {
    c.nseg = nseg;
    c.nrec = (int64_t)rec.size();
    c.max_len = 0;
    for (int64_t k = 0; k < nseg; ++k) c.max_len = std::max(c.max_len, off[k + 1] - off[k]);
    c.off = dev_alloc<int64_t>(nseg + 1);
    HIP_CHECK(hipMemcpy(c.off, off.data(), (nseg + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
    c.rec = dev_alloc<uint2>(rec.size());
    if (!rec.empty()) HIP_CHECK(hipMemcpy(c.rec, rec.data(), rec.size() * sizeof(uint2), hipMemcpyHostToDevice));
    c.off_h = std::move(off);
    build_tasks(g, c);
}


// Locality order of the segments of a Majorana graph.  Every record of a
// quadratic target {a, b} (beyond the quadratic x quadratic ones) pairs T+a with
// T+b, and every record of a quartic target K pairs a quadratic string with a
// quartic string sharing three modes T with K; in both cases the quartic
// operands of the record are rows T+w.  Each segment is sorted (stably) by the
// lexicographic rank of T, so the same position of every quadratic target
// touches the same rows, and a quartic target's records fall into groups that
// each read the rows of one triple.  Only the order of each sum changes.
// Returns whether every quartic target has 4 equal groups (its 4 triples).
static bool locality_order(const HostGraph& hg, const int64_t* off, int64_t N, std::vector<uint2>& rec) {
    const int m = hg.hdr.size;
    bool groups = true;
    std::vector<std::pair<int64_t, uint2>> buf;
    for (int64_t k = 0; k < N; ++k) {
        const uint64_t K = hg.labels[k];
        const int deg = __builtin_popcountll(K);
        if (deg != 2 && deg != 4) {
            groups = false;
            continue;
        }
        buf.clear();
        for (int64_t e = off[k]; e < off[k + 1]; ++e) {
            const uint64_t Li = hg.labels[rec[e].x & 0xFFFFFFu], Lj = hg.labels[rec[e].y & 0xFFFFFFu];
            uint64_t T = 0;
            if (deg == 2) T = Li & Lj;
            else T = K & (__builtin_popcountll(Li) == 4 ? Li : Lj);
            buf.push_back({__builtin_popcountll(T) == 3 ? lex_rank3(T, m) : -1, rec[e]});
        }
        std::stable_sort(buf.begin(), buf.end(),
                         [](const std::pair<int64_t, uint2>& x, const std::pair<int64_t, uint2>& y) {
                             return x.first < y.first;
                         });
        for (int64_t e = off[k]; e < off[k + 1]; ++e) rec[e] = buf[e - off[k]].second;
        if (deg == 4 && groups) {
            // 4 groups of len/4 records, each with one key, keys ascending
            const int64_t len = off[k + 1] - off[k], q = len / 4;
            if (len == 0 || len % 4 != 0) {
                groups = false;
                continue;
            }
            for (int t = 0; t < 4 && groups; ++t) {
                const int64_t key = buf[t * q].first;
                if (key < 0 || (t > 0 && key <= buf[(t - 1) * q].first)) groups = false;
                for (int64_t r = t * q; r < (t + 1) * q && groups; ++r)
                    if (buf[r].first != key) groups = false;
            }
        }
    }
    return groups;
}

// Device record of factor c and operand rows a (left) and b (right), both below
// 2^24: the factor's bf16 bit pattern (exact for every int8 value) rides in the
// top bytes, high byte with a and low byte with b, so the kernels rebuild the
// FP32 factor with integer operations instead of a table lookup.
static inline uint2 pack_record(int8_t c, uint32_t a, uint32_t b) {
    const float f = (float)c;
    uint32_t bits;
    std::memcpy(&bits, &f, 4);
    const uint32_t h = bits >> 16;  // the low 16 bits are zero for |c| <= 256
    return make_uint2(((h >> 8) << 24) | a, ((h & 0xFFu) << 24) | b);
}

// Quadratic-target blocks (see QuadBlockPlan): built only if every quadratic
// target's records, in locality order, are its leading records followed by
// exactly the pairs (T+u, T+v), (T+v, T+u) for every triple T outside {u, v}
// in lexicographic order.  Anything else leaves the plan off.
static void build_quadblocks(Graph& g, const HostGraph& hg, const int64_t* off, const std::vector<uint2>& rec) {
    QuadBlockPlan& q = g.qb;
    q.release();
    const int m = hg.hdr.size;
    const int64_t N = hg.hdr.n_ops;
    if (m < 5 || m > 64) return;
    std::unordered_map<uint64_t, int32_t> idx;
    idx.reserve((size_t)N * 2);
    for (int64_t k = 0; k < N; ++k) idx.emplace(hg.labels[k], (int32_t)k);
    std::vector<int32_t> qrow((size_t)m * m, -1);
    for (int64_t k = 0; k < N; ++k) {
        const uint64_t L = hg.labels[k];
        if (__builtin_popcountll(L) != 2) continue;
        const int u = __builtin_ctzll(L), v = __builtin_ctzll(L & (L - 1));
        if (v >= m) return;
        qrow[(size_t)u * m + v] = (int32_t)k;
    }
    for (int u = 0; u < m; ++u)
        for (int v = u + 1; v < m; ++v)
            if (qrow[(size_t)u * m + v] < 0) return;
    std::vector<uint64_t> tm;
    for (int a = 0; a < m; ++a)
        for (int b = a + 1; b < m; ++b)
            for (int d = b + 1; d < m; ++d) tm.push_back((1ull << a) | (1ull << b) | (1ull << d));
    const int64_t ntrip = (int64_t)tm.size();
    std::vector<int32_t> row4((size_t)ntrip * m, -1);
    for (int64_t t = 0; t < ntrip; ++t)
        for (int w = 0; w < m; ++w) {
            if (tm[t] >> w & 1) continue;
            const auto it = idx.find(tm[t] | (1ull << w));
            if (it == idx.end()) return;
            row4[(size_t)t * m + w] = it->second;
        }
    std::vector<int32_t> lead(N, 0);
    const uint32_t M24 = 0xFFFFFFu;
    const int ng = (m + 7) / 8, nbp = ng * (ng + 1) / 2;
    std::vector<int32_t> bp_of((size_t)ng * ng, -1);
    for (int g1 = 0, b = 0; g1 < ng; ++g1)
        for (int g2 = g1; g2 < ng; ++g2) bp_of[(size_t)g1 * ng + g2] = b++;
    std::vector<uint32_t> sgn((size_t)nbp * 8 * ntrip, 0);
    uint32_t fbits = 0;  // FP32 bit pattern of the common magnitude
    auto factor_bits = [](const uint2& r) { return (r.x & 0xFF000000u) | ((r.y >> 24) << 16); };
    for (int u = 0; u < m; ++u)
        for (int v = u + 1; v < m; ++v) {
            const int32_t k = qrow[(size_t)u * m + v];
            int64_t e = off[k];
            while (e < off[k + 1] &&
                   __builtin_popcountll(hg.labels[rec[e].x & M24] & hg.labels[rec[e].y & M24]) != 3)
                ++e;
            lead[k] = (int32_t)(e - off[k]);
            const uint64_t uv = (1ull << u) | (1ull << v);
            uint32_t* sg = sgn.data() + ((size_t)bp_of[(size_t)(u / 8) * ng + v / 8] * 8 + u % 8) * ntrip;
            const int j = v % 8;
            for (int64_t t = 0; t < ntrip; ++t) {
                if (tm[t] & uv) continue;
                const uint32_t ru = (uint32_t)row4[(size_t)t * m + u], rv = (uint32_t)row4[(size_t)t * m + v];
                if (e + 2 > off[k + 1]) return;
                if ((rec[e].x & M24) != ru || (rec[e].y & M24) != rv) return;
                if ((rec[e + 1].x & M24) != rv || (rec[e + 1].y & M24) != ru) return;
                for (int h = 0; h < 2; ++h) {
                    const uint32_t fb = factor_bits(rec[e + h]);
                    if (fbits == 0) fbits = fb & 0x7FFFFFFFu;
                    if ((fb & 0x7FFFFFFFu) != fbits) return;  // one magnitude only
                    if (fb >> 31) sg[t] |= 1u << (2 * j + h);
                }
                e += 2;
            }
            if (e != off[k + 1]) return;
        }
    if (fbits == 0) return;
    q.m = m;
    q.ntrip = ntrip;
    q.ng = ng;
    q.nbp = nbp;
    std::memcpy(&q.fmag, &fbits, 4);
    // about 1024 workgroups (two rounds of two 8-wavefront groups per CU)
    q.nr = (int32_t)std::max<int64_t>(1, std::min<int64_t>(ntrip, (1024 + q.nbp - 1) / q.nbp));
    std::vector<int2> bp;
    for (int g1 = 0; g1 < q.ng; ++g1)
        for (int g2 = g1; g2 < q.ng; ++g2) bp.push_back(make_int2(8 * g1, 8 * g2));
    q.row4 = dev_alloc<int32_t>(row4.size());
    HIP_CHECK(hipMemcpy(q.row4, row4.data(), row4.size() * 4, hipMemcpyHostToDevice));
    q.tmask = dev_alloc<uint64_t>(tm.size());
    HIP_CHECK(hipMemcpy(q.tmask, tm.data(), tm.size() * 8, hipMemcpyHostToDevice));
    q.bpair = dev_alloc<int2>(bp.size());
    HIP_CHECK(hipMemcpy(q.bpair, bp.data(), bp.size() * sizeof(int2), hipMemcpyHostToDevice));
    q.sgn = dev_alloc<uint32_t>(sgn.size());
    HIP_CHECK(hipMemcpy(q.sgn, sgn.data(), sgn.size() * 4, hipMemcpyHostToDevice));
    q.qrow = std::move(qrow);
    q.lead = std::move(lead);
    q.ok = true;
}

// orientation 0 from the bundle; 1 and 2 by stable counting sort
static void build_copies(Graph& g, const HostGraph& hg, int w, bool adjoint) {
    const int64_t N = hg.hdr.n_ops;
    const int64_t E = w == 0 ? hg.hdr.n_records : hg.hdr.n_gen_records;
    const int64_t* off = hg.off[w];
    const int32_t* ri = hg.ri[w];
    const int32_t* rj = hg.rj[w];
    const int8_t* rc = hg.rc[w];
    {
        std::vector<uint2> rec((size_t)E);
        for (int64_t e = 0; e < E; ++e)
            rec[e] = pack_record(rc[e], (uint32_t)ri[e], (uint32_t)rj[e]);
        if (w == 0 && hg.hdr.algebra == CUT_ALG_MAJORANA) {
            g.triple_groups = locality_order(hg, off, N, rec);
            build_quadblocks(g, hg, off, rec);
        }
        upload_csr(g, g.csr[w][0], N, std::vector<int64_t>(off, off + N + 1), rec);
    }
    if (!adjoint) return;
    for (int o = 1; o <= 2; ++o) {
        const int32_t* key = o == 1 ? rj : ri;
        std::vector<int64_t> noff(N + 1, 0);
        for (int64_t e = 0; e < E; ++e) noff[key[e] + 1]++;
        for (int64_t k = 0; k < N; ++k) noff[k + 1] += noff[k];
        std::vector<int64_t> cur(noff.begin(), noff.end() - 1);
        std::vector<uint2> rec((size_t)E);
        for (int64_t k = 0; k < N; ++k)
            for (int64_t e = off[k]; e < off[k + 1]; ++e) {
                if (o == 1) rec[cur[rj[e]]++] = pack_record(rc[e], (uint32_t)ri[e], (uint32_t)k);
                else rec[cur[ri[e]]++] = pack_record(rc[e], (uint32_t)k, (uint32_t)rj[e]);
            }
        upload_csr(g, g.csr[w][o], N, std::move(noff), rec);
    }
}

// Device record of a factor piece f, a value of at most 8 significant bits in
// the normal FP32 range: its bf16 bit pattern (the high half of f's FP32 bits,
// the low half being zero) rides in the top bytes as in pack_record.
static uint2 pack_piece(float f, uint32_t a, uint32_t b) {
    uint32_t bits;
    std::memcpy(&bits, &f, 4);
    const uint32_t h = bits >> 16;
    return make_uint2(((h >> 8) << 24) | a, ((h & 0xFFu) << 24) | b);
}

// Factor pieces.  A device record carries 8 significant bits of factor, so a
// wider factor v (Pauli-boson normal ordering reaches 24! C(48, 24) ~ 2e37 in
// the degree-24 one-mode registry) becomes several records on the same rows:
// piece t is the current remainder truncated to its leading 8 bits, and the
// remainder minus t is exact in FP64 and 8 bits shorter, so the pieces (at most
// 7 for an FP64 factor, 1 for any factor of <= 8 significant bits) all carry
// v's sign and sum exactly to v.  A piece outside the normal FP32 range is
// refused.  Returns the number of pieces.
static int factor_pieces(double v, float out[8]) {
    if (v == 0.0) return 0;
    {
        // the common case: a factor of <= 8 significant bits is its own piece
        const float f = (float)v;
        uint32_t bits;
        std::memcpy(&bits, &f, 4);
        const uint32_t ex = (bits >> 23) & 0xFFu;
        if ((double)f == v && (bits & 0xFFFFu) == 0 && ex != 0 && ex != 0xFFu) {
            out[0] = f;
            return 1;
        }
    }
    if (!std::isfinite(v)) CUT_FAIL(CUT_E_FORMAT, "factor %g is not finite", v);
    int n = 0;
    while (v != 0.0) {
        int e;
        const double m = std::frexp(v, &e);                         // v = m 2^e, 0.5 <= |m| < 1
        const double t = std::ldexp(std::trunc(std::ldexp(m, 8)), e - 8);
        if (e < -125 || e > 128 || n == 8)
            CUT_FAIL(CUT_E_UNSUPPORTED, "factor %.17g is outside the range of the device records", v);
        out[n++] = (float)t;                                         // exact: 8 significant bits
        v -= t;                                                      // exact
    }
    return n;
}

// Complex factor of record e of Pauli-boson record set w: int16 or FP64 pairs.
static inline void pb_factor(const HostGraph& hg, int w, int64_t e, double& re, double& im) {
    if (hg.hdr.factor_bytes == 16) {
        std::memcpy(&re, hg.rc[w] + 16 * e, 8);
        std::memcpy(&im, hg.rc[w] + 16 * e + 8, 8);
    } else {
        int16_t r, i;
        std::memcpy(&r, hg.rc[w] + 4 * e, 2);
        std::memcpy(&i, hg.rc[w] + 4 * e + 2, 2);
        re = r;
        im = i;
    }
}

// Uploads a target-grouped stream as orientation 0 of record set w and, with
// `adjoint`, the copies grouped by the right input (orientation 1: a kept,
// b := target; nb segments) and by the left input (orientation 2: a := target,
// b kept; na segments), each by a stable counting sort.
static void upload_set(Graph& g, int w, std::vector<int64_t>&& off, std::vector<uint2>&& rec, bool adjoint,
                       int64_t na, int64_t nb) {
    const int64_t nseg = (int64_t)off.size() - 1, E = (int64_t)rec.size();
    const int64_t rows = std::max(nseg, std::max(na, nb));
    if (adjoint) {
        for (int o = 1; o <= 2; ++o) {
            const int64_t ns = o == 1 ? nb : na;
            std::vector<int64_t> noff(ns + 1, 0);
            for (int64_t e = 0; e < E; ++e) noff[(o == 1 ? (rec[e].y & 0xFFFFFFu) : (rec[e].x & 0xFFFFFFu)) + 1]++;
            for (int64_t k = 0; k < ns; ++k) noff[k + 1] += noff[k];
            std::vector<int64_t> cur(noff.begin(), noff.end() - 1);
            std::vector<uint2> r2((size_t)E);
            for (int64_t k = 0; k < nseg; ++k)
                for (int64_t e = off[k]; e < off[k + 1]; ++e) {
                    const uint2 r = rec[e];
                    if (o == 1) r2[cur[r.y & 0xFFFFFFu]++] = make_uint2(r.x, (r.y & 0xFF000000u) | (uint32_t)k);
                    else r2[cur[r.x & 0xFFFFFFu]++] = make_uint2((r.x & 0xFF000000u) | (uint32_t)k, r.y);
                }
            upload_csr(g, g.csr[w][o], ns, std::move(noff), r2);
            g.csr[w][o].rows = rows;
        }
    }
    upload_csr(g, g.csr[w][0], nseg, std::move(off), rec);
    g.csr[w][0].rows = rows;
}

// Real-split form of a set of complex records (Pauli-boson graphs): a complex
// coefficient vector v of n entries is stored as 2n real rows, interleaved:
// row 2r = Re v_r, row 2r + 1 = Im v_r (the two halves of one coefficient
// share a cache line, so every gather of a complex record touches one line per
// operand).  A record y_k += c xi_a x_j with c = re + i im becomes
//   Re y_k += re (xi_a^r x_j^r - xi_a^i x_j^i) - im (xi_a^r x_j^i + xi_a^i x_j^r)
//   Im y_k += re (xi_a^r x_j^i + xi_a^i x_j^r) + im (xi_a^r x_j^r - xi_a^i x_j^i)
// i.e. up to four real records per target row and factor piece, kept in the
// stored order.
static void real_split(const HostGraph& hg, int w, int64_t nk, std::vector<int64_t>& off2, std::vector<uint2>& rec2) {
    const int64_t* off = hg.off[w];
    const int32_t* ri = hg.ri[w];
    const int32_t* rj = hg.rj[w];
    off2.assign(2 * nk + 1, 0);
    float pre[8], pim[8];
    for (int64_t k = 0; k < nk; ++k) {
        int64_t n = 0;
        for (int64_t e = off[k]; e < off[k + 1]; ++e) {
            double re, im;
            pb_factor(hg, w, e, re, im);
            n += 2 * factor_pieces(re, pre) + 2 * factor_pieces(im, pim);
        }
        off2[2 * k + 1] = n;    // real row of target k
        off2[2 * k + 2] = n;    // imaginary row (same count)
    }
    for (int64_t r = 0; r < 2 * nk; ++r) off2[r + 1] += off2[r];
    rec2.resize((size_t)off2[2 * nk]);
    for (int64_t k = 0; k < nk; ++k) {
        int64_t pr = off2[2 * k], pi = off2[2 * k + 1];
        for (int64_t e = off[k]; e < off[k + 1]; ++e) {
            double re, im;
            pb_factor(hg, w, e, re, im);
            const int nre = factor_pieces(re, pre), nim = factor_pieces(im, pim);
            const uint32_t ar = 2u * (uint32_t)ri[e], ai = ar + 1u;
            const uint32_t jr = 2u * (uint32_t)rj[e], ji = jr + 1u;
            for (int t = 0; t < nre; ++t) {
                rec2[pr++] = pack_piece(pre[t], ar, jr);
                rec2[pr++] = pack_piece(-pre[t], ai, ji);
                rec2[pi++] = pack_piece(pre[t], ar, ji);
                rec2[pi++] = pack_piece(pre[t], ai, jr);
            }
            for (int t = 0; t < nim; ++t) {
                rec2[pr++] = pack_piece(-pim[t], ar, ji);
                rec2[pr++] = pack_piece(-pim[t], ai, jr);
                rec2[pi++] = pack_piece(pim[t], ar, jr);
                rec2[pi++] = pack_piece(-pim[t], ai, ji);
            }
        }
    }
}

// Pauli-boson graph: every record set in real-split form; operator rows 2N,
// generator rows 2NG, outside rows 2Nc.
// Complex form of a set of records (Pauli-boson graphs), grouped by complex
// target in the stored order: x = (f_hi << 24) | (imag << 23) | a,
// y = (f_lo << 24) | j with (f_hi, f_lo) the bf16 pattern of a factor piece of
// the real or the imaginary part (one record per nonzero part and piece: the
// commutators of this algebra give purely real or purely imaginary factors).
// The left index must fit in 23 bits.
static void complex_records(const HostGraph& hg, int w, int64_t nk, std::vector<int64_t>& off2,
                            std::vector<uint2>& rec2) {
    const int64_t* off = hg.off[w];
    const int32_t* ri = hg.ri[w];
    const int32_t* rj = hg.rj[w];
    off2.assign(nk + 1, 0);
    float pre[8], pim[8];
    for (int64_t k = 0; k < nk; ++k) {
        int64_t n = 0;
        for (int64_t e = off[k]; e < off[k + 1]; ++e) {
            double re, im;
            pb_factor(hg, w, e, re, im);
            n += factor_pieces(re, pre) + factor_pieces(im, pim);
        }
        off2[k + 1] = off2[k] + n;
    }
    rec2.resize((size_t)off2[nk]);
    int64_t q = 0;
    for (int64_t e = 0; e < off[nk]; ++e) {
        double re, im;
        pb_factor(hg, w, e, re, im);
        if ((uint32_t)ri[e] >= (1u << 23))
            CUT_FAIL(CUT_E_UNSUPPORTED, "generator registry of %d labels exceeds 2^23", ri[e] + 1);
        const int nre = factor_pieces(re, pre), nim = factor_pieces(im, pim);
        for (int t = 0; t < nre; ++t) rec2[q++] = pack_piece(pre[t], (uint32_t)ri[e], (uint32_t)rj[e]);
        for (int t = 0; t < nim; ++t) {
            const uint2 r = pack_piece(pim[t], (uint32_t)ri[e], (uint32_t)rj[e]);
            rec2[q++] = make_uint2(r.x | (1u << 23), r.y);
        }
    }
}

static void load_pauli_boson(Graph& g, const HostGraph& hg, bool adjoint) {
    const int64_t N = hg.hdr.n_ops, NG = hg.n_gen;
    std::vector<int64_t> off;
    std::vector<uint2> rec;
    real_split(hg, 0, N, off, rec);                        // E_L: target k, left a (generator), right j
    upload_set(g, 0, std::move(off), std::move(rec), adjoint, 2 * NG, 2 * N);
    complex_records(hg, 0, N, off, rec);
    upload_csr(g, g.cxs[0], N, std::move(off), rec);
    g.cxs[0].na = NG;
    g.cxs[0].nb = N;
    g.csr[0][0].cx = &g.cxs[0];
    real_split(hg, 1, NG, off, rec);                       // E_eta: target a, left i, right j (operators)
    upload_set(g, 1, std::move(off), std::move(rec), adjoint, 2 * N, 2 * N);
    complex_records(hg, 1, NG, off, rec);
    upload_csr(g, g.cxs[1], NG, std::move(off), rec);
    g.cxs[1].na = N;
    g.cxs[1].nb = N;
    g.csr[1][0].cx = &g.cxs[1];
    if (hg.off[2]) {
        const int64_t Nc = hg.hdr.n_out_ops;
        real_split(hg, 2, Nc, off, rec);
        upload_set(g, 2, std::move(off), std::move(rec), false, 2 * NG, 2 * N);
        complex_records(hg, 2, Nc, off, rec);
        upload_csr(g, g.cxs[2], Nc, std::move(off), rec);
        g.cxs[2].na = NG;
        g.cxs[2].nb = N;
        g.csr[2][0].cx = &g.cxs[2];
        g.have_outside = true;
        g.n_out = 2 * Nc;
    }
}

// G2 stencil: the E_L records of target S whose left input is a pair coordinate
// P_a (the Wegner terms of the quadratic diagonal part), at most 4 per target.
static void build_stencil(Graph& g, const HostGraph& hg, const uint8_t* code) {
    const int64_t N = hg.hdr.n_ops, np = hg.hdr.n_pairs;
    std::vector<int32_t> pair_of(N, -1);
    for (int64_t a = 0; a < np; ++a) pair_of[hg.pairs[a]] = (int32_t)a;
    std::vector<int4> st((size_t)N * 4, make_int4(-1, 0, 0, 0));
    const int64_t* off = hg.off[0];
    for (int64_t S = 0; S < N; ++S) {
        int n = 0;
        for (int64_t e = off[S]; e < off[S + 1]; ++e) {
            const int32_t a = pair_of[hg.ri[0][e]];
            if (a < 0) continue;
            if (n == 4) return;  // not a pair-flip algebra: no G2 stencil
            st[S * 4 + n++] = make_int4(hg.rj[0][e], a, code[(uint8_t)hg.rc[0][e]], 0);
        }
    }
    // transposed stencil (by partner row) and per-pair lists, in (S, t) order
    std::vector<int64_t> toff(N + 1, 0), poff(np + 1, 0);
    for (int64_t q = 0; q < N * 4; ++q)
        if (st[q].x >= 0) {
            toff[st[q].x + 1]++;
            poff[st[q].y + 1]++;
        }
    for (int64_t r = 0; r < N; ++r) toff[r + 1] += toff[r];
    for (int64_t a = 0; a < np; ++a) poff[a + 1] += poff[a];
    std::vector<int4> tent(toff[N]), pent(poff[np]);
    std::vector<int64_t> tc(toff.begin(), toff.end() - 1), pc(poff.begin(), poff.end() - 1);
    for (int64_t S = 0; S < N; ++S)
        for (int t = 0; t < 4; ++t) {
            const int4 e = st[S * 4 + t];
            if (e.x < 0) break;
            tent[tc[e.x]++] = make_int4((int32_t)S, e.y, e.z, 0);
            pent[pc[e.y]++] = make_int4((int32_t)S, e.x, e.z, 0);
        }
    g.stencil = dev_alloc<int4>(st.size());
    HIP_CHECK(hipMemcpy(g.stencil, st.data(), st.size() * sizeof(int4), hipMemcpyHostToDevice));
    g.st_t_off = dev_alloc<int64_t>(N + 1);
    HIP_CHECK(hipMemcpy(g.st_t_off, toff.data(), (N + 1) * 8, hipMemcpyHostToDevice));
    g.st_t = dev_alloc<int4>(tent.size());
    if (!tent.empty()) HIP_CHECK(hipMemcpy(g.st_t, tent.data(), tent.size() * sizeof(int4), hipMemcpyHostToDevice));
    g.st_p_off = dev_alloc<int64_t>(np + 1);
    HIP_CHECK(hipMemcpy(g.st_p_off, poff.data(), (np + 1) * 8, hipMemcpyHostToDevice));
    g.st_p = dev_alloc<int4>(pent.size());
    if (!pent.empty()) HIP_CHECK(hipMemcpy(g.st_p, pent.data(), pent.size() * sizeof(int4), hipMemcpyHostToDevice));
    g.have_stencil = true;
}

}  // namespace cut

using namespace cut;

extern "C" const char* cut_last_error(void) { return g_err; }
extern "C" const char* cut_version(void) { return "cutgraph 1.0 gfx950"; }

extern "C" cut_status cut_graph_load(const char* path, int32_t dev, uint32_t flags, cut_graph_t* out) {
    Graph* g = nullptr;
    int prev = 0;
    bool switched = false;
    try {
        if (!path || !out) CUT_FAIL(CUT_E_INVAL, "cut_graph_load: null argument");
        *out = nullptr;
        HostGraph hg;
        read_bundle(path, (flags & CUT_LOAD_NO_CHECKSUM) == 0, hg);
        const int64_t N = hg.hdr.n_ops;
        const bool pb = hg.hdr.algebra == CUT_ALG_PAULI_BOSON;
        if (pb != (hg.hdr.factor_bytes == 4 || hg.hdr.factor_bytes == 16) || pb != (hg.hdr.n_gen_ops > 0))
            CUT_FAIL(CUT_E_FORMAT, "%s: factor format does not match the algebra", path);
        const int64_t rows = pb ? 2 * N : N, grows = pb ? 2 * hg.n_gen : N;
        if (rows >= (1ll << 24) || grows >= (1ll << 24) || (pb && 2 * hg.hdr.n_out_ops >= (1ll << 31)))
            CUT_FAIL(CUT_E_UNSUPPORTED, "registry of %lld rows exceeds 2^24", (long long)std::max(rows, grows));
        // factor dictionary over the int8 record sets (G2 stencil tables)
        uint8_t code[256];
        std::memset(code, 0, sizeof code);
        std::vector<double> ftab;
        if (!pb) {
            bool seen[256] = {false};
            for (int w = 0; w < 3; ++w) {
                const int64_t E = w == 0 ? hg.hdr.n_records : w == 1 ? hg.hdr.n_gen_records : hg.hdr.n_out_records;
                for (int64_t e = 0; e < E; ++e) seen[(uint8_t)hg.rc[w][e]] = true;
            }
            for (int v = -128; v < 128; ++v)
                if (seen[(uint8_t)v]) {
                    code[(uint8_t)v] = (uint8_t)ftab.size();
                    ftab.push_back((double)v);
                }
        }
        HIP_CHECK(hipGetDevice(&prev));
        HIP_CHECK(hipSetDevice(dev));
        switched = true;
        g = new Graph();
        g->device = dev;
        g->hdr = hg.hdr;
        g->N = rows;
        g->NG = grows;
        g->gen_sign = hg.hdr.gen_sign;
        g->nfactors = (int)ftab.size();
        // factor dictionary of the G2 stencil tables (the record streams carry
        // their factors themselves)
        g->ftab = dev_alloc<double>(256);
        ftab.resize(256, 0.0);
        HIP_CHECK(hipMemcpy(g->ftab, ftab.data(), 256 * sizeof(double), hipMemcpyHostToDevice));
        const bool adj = (flags & CUT_LOAD_ADJOINT) != 0;
        g->labels_h.assign(hg.labels, hg.labels + N);
        if (hg.gen_labels) g->gen_labels_h.assign(hg.gen_labels, hg.gen_labels + hg.n_gen);
        if (hg.out_labels) g->out_labels_h.assign(hg.out_labels, hg.out_labels + hg.hdr.n_out_ops);
        g->have_adjoint = adj;
        if (pb) {
            load_pauli_boson(*g, hg, adj);
        } else {
            build_copies(*g, hg, 0, adj);
            build_copies(*g, hg, 1, adj);
            if (hg.off[2]) {
                // outside-space records: target order only, segments = outside rows
                const int64_t Nc = hg.hdr.n_out_ops, Ec = hg.hdr.n_out_records;
                std::vector<uint2> rec((size_t)Ec);
                for (int64_t e = 0; e < Ec; ++e)
                    rec[e] = pack_record(hg.rc[2][e], (uint32_t)hg.ri[2][e], (uint32_t)hg.rj[2][e]);
                upload_csr(*g, g->csr[2][0], Nc, std::vector<int64_t>(hg.off[2], hg.off[2] + Nc + 1), rec);
                g->have_outside = true;
                g->n_out = Nc;
            }
            g->diag = dev_alloc<uint8_t>(N);
            HIP_CHECK(hipMemcpy(g->diag, hg.diag, N, hipMemcpyHostToDevice));
            g->npairs = hg.hdr.n_pairs;
            g->pairs = dev_alloc<int32_t>(g->npairs);
            if (g->npairs) HIP_CHECK(hipMemcpy(g->pairs, hg.pairs, g->npairs * 4, hipMemcpyHostToDevice));
            build_stencil(*g, hg, code);
        }
        {
            int lds = 0;
            if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && lds > 0)
                g->max_lds = lds;
        }
        if (!pb) build_tiles(*g, hg, code);
        HIP_CHECK(hipDeviceSynchronize());
        HIP_CHECK(hipSetDevice(prev));
        *out = (cut_graph_t)g;
        return CUT_OK;
    } catch (const Fail& f) {
        delete g;
        if (switched) (void)hipSetDevice(prev);
        return f.st;
    } catch (const std::bad_alloc&) {
        delete g;
        if (switched) (void)hipSetDevice(prev);
        set_error("cut_graph_load: out of host memory");
        return CUT_E_NOMEM;
    }
}

extern "C" void cut_graph_free(cut_graph_t h) { delete (Graph*)h; }

extern "C" cut_status cut_graph_info(cut_graph_t h, cut_graph_desc* d) {
    if (!h || !d) {
        set_error("cut_graph_info: null argument");
        return CUT_E_INVAL;
    }
    const Graph& g = *(const Graph*)h;
    std::memset(d, 0, sizeof *d);
    d->algebra = g.hdr.algebra;
    d->size = g.hdr.size;
    d->n_ops = g.hdr.n_ops;
    d->n_records = g.hdr.n_records;
    d->n_gen_records = g.hdr.n_gen_records;
    d->n_pairs = g.hdr.n_pairs;
    d->n_out_ops = g.hdr.n_out_ops;
    d->n_out_records = g.hdr.n_out_records;
    d->n_gen_ops = g.hdr.n_gen_ops;
    d->checksum = g.hdr.records_checksum;
    d->file_bytes = (int64_t)g.hdr.file_bytes;
    std::strncpy(d->identifier, g.hdr.identifier, sizeof d->identifier - 1);
    return CUT_OK;
}

extern "C" cut_status cut_graph_labels(cut_graph_t h, int32_t which, uint64_t* out, int64_t n) {
    if (!h || !out) {
        set_error("cut_graph_labels: null argument");
        return CUT_E_INVAL;
    }
    const Graph& g = *(const Graph*)h;
    const std::vector<uint64_t>* v = which == CUT_GRAPH_FLOW ? &g.labels_h
                                     : which == CUT_GRAPH_GEN ? (g.gen_labels_h.empty() ? &g.labels_h : &g.gen_labels_h)
                                     : which == CUT_GRAPH_OUTSIDE ? &g.out_labels_h : nullptr;
    if (!v || (which == CUT_GRAPH_OUTSIDE && !g.have_outside)) {
        set_error("cut_graph_labels: unknown or absent registry %d", which);
        return CUT_E_INVAL;
    }
    if (n != (int64_t)v->size()) {
        set_error("cut_graph_labels: registry %d has %lld labels, %lld requested", which, (long long)v->size(),
                  (long long)n);
        return CUT_E_INVAL;
    }
    std::memcpy(out, v->data(), v->size() * sizeof(uint64_t));
    return CUT_OK;
}

extern "C" cut_status cut_graph_set_tiling(cut_graph_t h, int64_t long_records, int64_t chunk_records,
                                           uint32_t flags) {
    try {
        if (!h || long_records < 1 || chunk_records < 1 || (flags & ~127u))
            CUT_FAIL(CUT_E_INVAL, "cut_graph_set_tiling: bad argument");
        Graph& g = *(Graph*)h;
        DeviceGuard dg(g.device);
        HIP_CHECK(hipDeviceSynchronize());
        apply_tiling(g, long_records, chunk_records, flags);
        rereserve(g);
        return CUT_OK;
    } catch (const Fail& f) {
        return f.st;
    }
}
