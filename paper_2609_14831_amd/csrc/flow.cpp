// Flow driver: classic RK4 coflow of H and its observables (Sec. 2.1 Eq. coflow;
// Sec. 2.4 Eq. forward-coeff) and the exact adjoint of the discrete RK4 map.
//
// One RK step = 4 x { generator eta(h) ; graph pass with the fused RK stage
// epilogue }, then a device step counter is bumped.  Per-set activity
// (t < n_steps[s]) is read on the device from that counter, so the same
// kernel sequence serves every step and is captured once as a hipGraph.
//
// Work area (reserved with cut_graph_reserve, kept in the handle):
//   xsh[2]  next/current stage operand (float or double) [N][nops][nsets]
//   acc     RK accumulator (double)                     [N][nops][nsets]
//   hst     FP64 Hamiltonian column of the stage         [N][nsets]
//   eta     generator in the stage precision              [N][nsets]
//   nsteps, step, flag (int32)
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "internal.h"

namespace cut {

// Captured RK steps of one flow configuration (key), one graph per width
// class: the sets a step launches over (0 = all of them, else the active
// prefix length, see set_ranges).  Replays run on `stream`; captures are made
// on `cap`, which never runs work.
struct StepGraphCache {
    struct Cls {
        int64_t id;
        hipGraph_t graph;
        hipGraphExec_t exec;
    };
    std::vector<Cls> cls;
    hipStream_t stream = nullptr, cap = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    std::vector<uint64_t> key;
};

void release_step_graphs(Graph& g) {
    StepGraphCache* c = g.graphs;
    if (!c) return;
    for (auto& e : c->cls) {
        if (e.exec) (void)hipGraphExecDestroy(e.exec);
        if (e.graph) (void)hipGraphDestroy(e.graph);
    }
    if (c->ev_in) (void)hipEventDestroy(c->ev_in);
    if (c->ev_out) (void)hipEventDestroy(c->ev_out);
    if (c->stream) (void)hipStreamDestroy(c->stream);
    if (c->cap) (void)hipStreamDestroy(c->cap);
    delete c;
    g.graphs = nullptr;
}

// Launch pieces covering the sets [0, A).  A piece of w sets runs with lane
// groups of w lanes (w a power of two), and its pass costs a fixed part (the
// record stream, the per-record decode, the combine) plus the cache lines its
// gathers touch: in the layout of all the sets one per operand and line-sized
// group of sets, so pieces of 8 to 32 sets cost about the same.  Measured on
// the 2n = 40 graph, 64 sets x 5 operands, F32C, per RK step, in one session:
// 21-27 active sets 5.1 ms as one piece of 32 sets; 39-41 active sets 10.3 ms
// as pieces of 32 + the rest, 10.05 ms as one full-width launch (which keeps
// the tiling's block kernels).  Cover: pieces of 64 sets while more than 32
// remain, then one piece of the rest.  Prefixes of 16 sets or fewer are
// compacted instead (compact_width).
struct SetRange {
    int32_t s0, s1;
};
static std::vector<SetRange> set_ranges(int32_t A) {
    std::vector<SetRange> r;
    int32_t s = 0;
    while (A - s > 32) {
        const int32_t n = std::min(64, A - s);
        r.push_back({s, s + n});
        s += n;
    }
    if (A > s) r.push_back({s, A});
    return r;
}

// Widest compacted state, and widest phase whose full-width passes take the
// segment kernel (lane groups of <= 16 sets) instead of the tiling's block and
// tile kernels.
static const int32_t kCompactSets = 16;
static const int32_t kNarrowSets = 16;

// Sets the flow's state carries while A sets are still active.  Once the
// active prefix fits in 16 sets, the finished sets' columns are written out
// and the state, stage operands and Hamiltonian column are repacked into the
// layout of W sets, W the smallest power of two >= A.  In the layout of all
// the sets every operand's few active sets sit on a cache line of their own,
// so a pass over 16 sets or fewer reads as many lines per row as one over 32;
// repacked, a row's active sets are contiguous.  Wider states do not pay: a
// state repacked to 32 sets measured slower than a 32-set piece of the full
// layout (5.18 against 5.10 ms per RK step at 21-27 active sets, 6.33 against
// 5.07 at 32, where its full-width passes take the block kernels), and widths
// that are not powers of two put operand runs across cache lines (a 55-set
// state took 14.3 against 10.3 ms per RK step).
static int32_t compact_width(int32_t A, int32_t nsets) {
    if (A > kCompactSets) return nsets;
    int32_t W = 1;
    while (W < A) W <<= 1;
    return std::min(W, nsets);
}

static size_t al(size_t x) { return (x + 255) & ~size_t(255); }

struct FlowBufs {
    void* xsh[2];
    double* acc;
    double* hst;
    void* eta;
    int32_t* nsteps;
    int32_t* step;
    int32_t* flag;
    double* part;   // tile partial slots (null when the tile path is not taken)
    double* zp;     // the state with its sets in flow order (see cut_flow_integrate)
    int32_t* perm;  // flow order: position q holds caller set perm[q]
};

// byte offsets of the flow's work area (one layout for sizing and carving)
struct FlowLayout {
    size_t xs0, xs1, acc, hst, eta, ns, st, fl, part, zp, perm, ex, total, part_bytes;
};

static FlowLayout flow_layout(const Graph& g, int64_t nsets, int64_t nops, int prec, size_t extra) {
    const bool f32 = prec != CUT_F64;
    FlowLayout L{};
    L.part_bytes = forward_partial_bytes(g, (int32_t)nsets, (int32_t)nops, prec);
    const int64_t N = g.N, cols = nops * nsets;
    const size_t tb = f32 ? 4 : 8;
    size_t o = 0;
    L.xs0 = o;
    o += al(N * cols * tb);
    L.xs1 = o;
    o += al(N * cols * tb);
    L.acc = o;
    o += al(N * cols * 8);
    L.hst = o;
    o += al(N * nsets * 8);
    L.eta = o;
    o += al(g.NG * nsets * tb);
    L.ns = o;
    o += al(nsets * 4);
    L.st = o;
    o += 256;
    L.fl = o;
    o += 256;
    L.part = o;
    o += al(L.part_bytes);
    L.zp = o;
    o += al(N * cols * 8);
    L.perm = o;
    o += al(nsets * 4);
    L.ex = o;
    o += al(extra);
    L.total = o;
    return L;
}

size_t flow_ws_bytes(const Graph& g, int64_t nsets, int64_t nops, int prec, size_t extra) {
    return flow_layout(g, nsets, nops, prec, extra).total;
}

size_t flow_outside_extra(const Graph& g, int64_t nsets, int64_t nops) {
    const int64_t cols = nops * nsets;
    // outside action, partial sums of its squares, the accumulated norms in flow order
    return g.have_outside ? al(g.n_out * cols * 8) + al((size_t)kColsqParts * cols * 8) + al(cols * 8) : 0;
}

// stage storage, zr, lam_new, mu, u, eta, geta, vjp scratch of the adjoint flow
size_t flow_adjoint_extra(const Graph& g, int64_t nsets, int64_t nops, int64_t ckpt_every) {
    const int64_t M = g.N * nops * nsets;
    const int64_t nslot = ckpt_every * 4 + 1;
    return al(nslot * M * 8) + 4 * al(M * 8) + 2 * al(g.NG * nsets * 8) + al(2 * g.N * nsets * 8);
}

static FlowBufs flow_bufs(Graph& g, int64_t nsets, int64_t nops, int prec, size_t extra, char** extra_ptr) {
    const FlowLayout L = flow_layout(g, nsets, nops, prec, extra);
    char* b = (char*)g.ws.need(L.total, extra > 0 ? "the flow (with its diagnostic or adjoint storage)" : "the flow");
    FlowBufs f;
    f.xsh[0] = b + L.xs0;
    f.xsh[1] = b + L.xs1;
    f.acc = (double*)(b + L.acc);
    f.hst = (double*)(b + L.hst);
    f.eta = b + L.eta;
    f.nsteps = (int32_t*)(b + L.ns);
    f.step = (int32_t*)(b + L.st);
    f.flag = (int32_t*)(b + L.fl);
    f.part = L.part_bytes ? (double*)(b + L.part) : nullptr;
    f.zp = (double*)(b + L.zp);
    f.perm = (int32_t*)(b + L.perm);
    if (extra_ptr) *extra_ptr = b + L.ex;
    return f;
}

struct StepPlan {
    Graph* g;
    int gen;
    int prec;
    double ds, delta;
    int32_t nsets, nops;
    FlowBufs fb;
    double* z;
    // stage operand pointers: stage s reads xin[s], writes xout[s]
    void* xin[4];
    void* xout[4];
    // outside-space diagnostic (null when off): accumulated column norms, the
    // stage's outside action [n_out][cols] and the partial sums of its squares
    double* onorm = nullptr;
    double* cbuf = nullptr;
    double* cpart = nullptr;
    // sets each graph pass launches over (empty: all of them in one launch)
    std::vector<SetRange> ranges;
    // the state is a compacted phase of at most kNarrowSets sets: full-width
    // passes take the segment kernel
    int32_t narrow = 0;
    // narrowest lane group: that of the layout of all the sets, so that a
    // compacted phase sums every term in the same order (bitwise the same flow)
    int32_t gfloor = 1;
};

// HIP events bracketing launches (kind 0 = graph pass, 1 = generator)
struct PassTimer {
    std::vector<hipEvent_t> ev;
    std::vector<int> kind;
    size_t used = 0;
    hipEvent_t next() {
        if (used == ev.size()) {
            hipEvent_t e;
            HIP_CHECK(hipEventCreate(&e));
            ev.push_back(e);
        }
        return ev[used++];
    }
    void mark(int k, hipStream_t s) {
        HIP_CHECK(hipEventRecord(next(), s));
        if (used % 2 == 1) kind.push_back(k);
    }
    ~PassTimer() {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
};

// the kernel sequence of one RK step (stream-ordered, capturable)
static void enqueue_step(const StepPlan& P, hipStream_t s, PassTimer* tm = nullptr) {
    Graph& g = *P.g;
    const bool f32 = P.prec != CUT_F64;
    const int64_t cols = (int64_t)P.nops * P.nsets;
    for (int st = 0; st < 4; ++st) {
        if (tm) tm->mark(1, s);
        eval_generator(g, P.gen, P.delta, P.nsets, P.fb.hst, P.nsets, P.fb.eta, P.nsets, f32, P.fb.nsteps,
                       P.fb.step, s);
        if (tm) tm->mark(1, s);
        if (P.onorm) {
            // C(eta_s, Z_s) over E_C, then b_s ds sum_q C_q^2 per column
            static const double b[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
            PassArgs c{};
            c.csr = &g.csr[2][0];
            c.A = P.fb.eta;
            c.lda = P.nsets;
            c.B = P.xin[st];
            c.ldb = cols;
            c.nsets = P.nsets;
            c.nops = P.nops;
            c.precision = P.prec;
            c.nsteps = P.fb.nsteps;
            c.step = P.fb.step;
            c.y = P.cbuf;
            c.ldy = cols;
            c.scale = 1.0;
            launch_pass(MODE_BCAST, EPI_Y, c, s);
            launch_colsq_accumulate(P.cbuf, g.n_out, cols, P.nsets, P.cpart, kColsqParts, P.fb.nsteps, P.fb.step,
                                    b[st] * P.ds, P.onorm, s);
        }
        PassArgs p{};
        p.csr = &g.csr[0][0];
        p.A = P.fb.eta;
        p.lda = P.nsets;
        p.B = P.xin[st];
        p.ldb = cols;
        p.nsets = P.nsets;
        p.nops = P.nops;
        p.precision = P.prec;
        p.nsteps = P.fb.nsteps;
        p.step = P.fb.step;
        p.stage = st;
        p.ds = P.ds;
        p.z = P.z;
        p.acc = P.fb.acc;
        p.xout = P.xout[st];
        p.hst = P.fb.hst;
        p.ldh = P.nsets;
        p.gmax = 64 >> g.bchunk;  // the tiling's B-chunk
        p.narrow = P.narrow;
        p.gfloor = P.gfloor;
        if (tm) tm->mark(0, s);
        const size_t nr = std::max<size_t>(1, P.ranges.size());
        for (size_t r = 0; r < nr; ++r) {
            if (!P.ranges.empty()) {
                p.s0 = P.ranges[r].s0;
                p.s1 = P.ranges[r].s1;
            }
            if (P.fb.part) launch_forward(g, EPI_RK, p, P.fb.part, s);
            else launch_pass(MODE_BCAST, EPI_RK, p, s);
        }
        if (tm) tm->mark(0, s);
    }
    launch_bump(P.fb.step, s);
}

static void check_flow(Graph& g, const cut_flow_params* p, int64_t nsets, int64_t nops, const int32_t* n_steps) {
    if (!p || !n_steps) CUT_FAIL(CUT_E_INVAL, "flow: null params or n_steps");
    check_prec(p->precision);
    check_shape(nsets, nops);
    check_generator(g, p->generator);
    if (!(p->ds > 0.0) || !std::isfinite(p->ds)) CUT_FAIL(CUT_E_INVAL, "flow: ds must be positive");
    if (p->ckpt_every < 0) CUT_FAIL(CUT_E_INVAL, "flow: ckpt_every < 0");
    for (int64_t s = 0; s < nsets; ++s)
        if (n_steps[s] < 0) CUT_FAIL(CUT_E_INVAL, "flow: negative n_steps");
}

}  // namespace cut

using namespace cut;

extern "C" cut_status cut_flow_integrate(cut_graph_t h, const cut_flow_params* p, int64_t nsets, int64_t nops,
                                         const int32_t* n_steps, double* z, double* ckpt, void* stream_) {
    try {
        Graph& g = checked(h);
        check_flow(g, p, nsets, nops, n_steps);
        if (!z) CUT_FAIL(CUT_E_INVAL, "flow: null state");
        DeviceGuard dg(g.device);
        hipStream_t stream = (hipStream_t)stream_;
        int64_t T = 0;
        for (int64_t s = 0; s < nsets; ++s) T = std::max<int64_t>(T, n_steps[s]);
        const int64_t t0 = std::max<int64_t>(0, p->step_begin);
        const int64_t t1 = p->step_end < 0 ? T : std::min<int64_t>(p->step_end, T);
        const bool f32 = p->precision != CUT_F64;
        const int64_t cols = nops * nsets, M = g.N * cols;
        const bool outside = p->outside_norm2 != nullptr;
        if (outside && !g.have_outside)
            CUT_FAIL(CUT_E_INVAL, "flow: outside_norm2 needs a graph with outside-space records");
        const size_t ob = outside ? flow_outside_extra(g, nsets, nops) : 0;
        char* oex = nullptr;
        FlowBufs fb = flow_bufs(g, nsets, nops, p->precision, ob, &oex);
        // Ragged batch: the sets run in the order of decreasing n_steps, so the
        // sets still active at step t are a prefix of length A(t) and each
        // graph pass launches over that prefix only (in pieces, set_ranges).
        // The state is permuted into that order in the work area and back at
        // the end (so are the outside-space diagnostic's accumulated columns),
        // and the passes are cut into the same pieces with or without the
        // diagnostic.
        std::vector<int32_t>& perm = g.flow_perm_h;
        std::vector<int32_t>& ns_run = g.flow_nsteps_h;
        perm.resize(nsets);
        for (int32_t q = 0; q < (int32_t)nsets; ++q) perm[q] = q;
        std::stable_sort(perm.begin(), perm.end(), [&](int32_t a, int32_t b) { return n_steps[a] > n_steps[b]; });
        bool identity = true;
        for (int32_t q = 0; q < (int32_t)nsets; ++q) identity = identity && perm[q] == q;
        ns_run.resize(nsets);
        for (int32_t q = 0; q < (int32_t)nsets; ++q) ns_run[q] = n_steps[perm[q]];
        auto active = [&](int64_t t) {
            int32_t A = 0;
            for (int32_t q = 0; q < (int32_t)nsets; ++q) A += ns_run[q] > t;
            return A;
        };
        // whether the passes over W sets honour set ranges (the segment kernel;
        // not the complex-record kernels, whose lanes are columns)
        auto ranged_at = [&](int32_t W) {
            PassArgs probe{};
            probe.csr = &g.csr[0][0];
            probe.nsets = W;
            probe.nops = (int32_t)nops;
            probe.precision = p->precision;
            probe.lda = W;
            probe.ldb = (int64_t)nops * W;
            return forward_set_ranges(g, probe);
        };
        // Compacted phases (compact_width): the state carries the active
        // prefix only, with the lane groups and so the sums of the full layout.
        // Not with the diagnostic (its columns keep the full layout),
        // checkpoints (full states in caller order) or passes that cover every
        // set.
        const bool compact = !outside && !(ckpt && p->ckpt_every > 0) && t1 > t0 && ranged_at((int32_t)nsets) &&
                             compact_width(active(t1 - 1), (int32_t)nsets) < nsets;
        auto phase_width = [&](int64_t t) -> int32_t {
            return compact ? compact_width(active(t), (int32_t)nsets) : (int32_t)nsets;
        };
        // the widths the state takes over [t0, t1), in order
        std::vector<int32_t> phases;
        for (int64_t t = t0; t < t1 && compact; ++t)
            if (phases.empty() || phases.back() != phase_width(t)) phases.push_back(phase_width(t));
        if (phases.empty()) phases.push_back((int32_t)nsets);
        double* zs = (identity && !compact) ? z : fb.zp;
        HIP_CHECK(hipMemcpyAsync(fb.nsteps, ns_run.data(), nsets * 4, hipMemcpyHostToDevice, stream));
        if (zs != z) {
            HIP_CHECK(hipMemcpyAsync(fb.perm, perm.data(), nsets * 4, hipMemcpyHostToDevice, stream));
            launch_move_sets(z, (int32_t)nsets, zs, phases[0], g.N, (int32_t)nops, 0, phases[0], fb.perm, false,
                             stream);
        }
        launch_set_scalar(fb.step, (int32_t)t0, stream);
        int32_t* const flagp = p->nonfinite ? p->nonfinite : fb.flag;
        launch_set_scalar(flagp, 0, stream);
        StepPlan P{&g, p->generator, p->precision, p->ds, p->delta, (int32_t)nsets, (int32_t)nops, fb, zs, {}, {}};
        for (int st = 0; st < 4; ++st) {
            P.xin[st] = fb.xsh[st & 1];
            P.xout[st] = fb.xsh[(st + 1) & 1];
        }
        if (outside) {
            P.cbuf = (double*)oex;
            P.cpart = (double*)(oex + al(g.n_out * cols * 8));
            P.onorm = p->outside_norm2;
            if (zs != z) {
                // the accumulated norms in flow order (one row of nops x nsets)
                P.onorm = (double*)(oex + al(g.n_out * cols * 8) + al((size_t)kColsqParts * cols * 8));
                launch_move_sets(p->outside_norm2, (int32_t)nsets, P.onorm, (int32_t)nsets, 1, (int32_t)nops, 0,
                                 (int32_t)nsets, fb.perm, false, stream);
            }
        }
        // phase k of a compacted flow keeps the state in zp (k even) or in
        // the RK accumulator's buffer (k odd), the accumulator in the other:
        // stage 0 of every step rewrites the accumulator, so at a step
        // boundary it holds nothing
        auto enter = [&](size_t k) {
            P.nsets = phases[k];
            P.narrow = (phases[k] < nsets && phases[k] <= kNarrowSets) ? 1 : 0;
            if (compact) {
                P.z = (k & 1) ? fb.acc : fb.zp;
                P.fb.acc = (k & 1) ? fb.zp : fb.acc;
            }
        };
        // lane groups of a launch over w sets of the full layout span
        // max(w, min(8, nsets)) sets rounded up to a power of two
        while (P.gfloor < std::min<int64_t>(8, nsets)) P.gfloor <<= 1;
        enter(0);
        launch_prep_state(P.z, g.N, (int32_t)nops, P.nsets, fb.xsh[0], f32, fb.hst, stream);
        // width class of step t: the sets up to the last active one, when the
        // pass honours set ranges (else 0: every set of the phase in one launch)
        // (a prefix that one 64-set piece would cover runs as a full-width
        // launch instead, which keeps the tiling's block and tile kernels)
        auto width_class = [&](int64_t t) -> int64_t {
            const int32_t W = phase_width(t);
            if (!ranged_at(W)) return 0;
            int64_t last = 0;
            for (int32_t q = 0; q < W; ++q)
                if (ns_run[q] > t) last = q + 1;
            if (last == W) return 0;
            const std::vector<SetRange> r = set_ranges((int32_t)last);
            if (W <= 64 && r.size() == 1 && r[0].s1 - r[0].s0 > 32) return 0;
            return last;
        };
        auto set_class = [&](int64_t c) {
            P.ranges.clear();
            if (c > 0) P.ranges = set_ranges((int32_t)c);
        };
        // captured step of phase k and class c (the phase's width and parity
        // fix the state's layout and buffers)
        auto graph_id = [&](size_t k, int64_t c) {
            return ((int64_t)phases[k] << 33) | ((int64_t)(k & 1) << 32) | c;
        };
        const bool use_graph = (p->flags & CUT_FLOW_HIPGRAPH) && t1 - t0 > 1;
        const bool timed = !use_graph && (p->flags & CUT_FLOW_TIME_PASSES);
        PassTimer timer;
        g.timing = cut_flow_timing{};
        StepGraphCache* gc = nullptr;
        if (use_graph) {
            std::vector<uint64_t> key = {(uint64_t)(uintptr_t)zs, (uint64_t)(uintptr_t)g.ws.ptr, (uint64_t)p->generator,
                                         (uint64_t)p->precision, (uint64_t)nsets, (uint64_t)nops, 0, 0,
                                         g.tiling_gen, (uint64_t)(uintptr_t)fb.part,
                                         (uint64_t)(uintptr_t)p->outside_norm2};
            std::memcpy(&key[6], &p->ds, 8);
            std::memcpy(&key[7], &p->delta, 8);
            if (!g.graphs || g.graphs->key != key) {
                release_step_graphs(g);
                gc = new StepGraphCache();
                g.graphs = gc;
                HIP_CHECK(hipStreamCreateWithFlags(&gc->stream, hipStreamNonBlocking));
                HIP_CHECK(hipStreamCreateWithFlags(&gc->cap, hipStreamNonBlocking));
                HIP_CHECK(hipEventCreateWithFlags(&gc->ev_in, hipEventDisableTiming));
                HIP_CHECK(hipEventCreateWithFlags(&gc->ev_out, hipEventDisableTiming));
                gc->key = key;
            }
            gc = g.graphs;
            // capture every (phase, width class) this call needs before any replay
            size_t k = 0;
            for (int64_t t = t0; t < t1; ++t) {
                if (phase_width(t) != phases[k]) ++k;
                const int64_t c = width_class(t), id = graph_id(k, c);
                bool have = false;
                for (auto& e : gc->cls) have = have || e.id == id;
                if (have) continue;
                enter(k);
                set_class(c);
                StepGraphCache::Cls e{id, nullptr, nullptr};
                HIP_CHECK(hipStreamBeginCapture(gc->cap, hipStreamCaptureModeThreadLocal));
                enqueue_step(P, gc->cap);
                HIP_CHECK(hipStreamEndCapture(gc->cap, &e.graph));
                HIP_CHECK(hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0));
                gc->cls.push_back(e);
            }
            enter(0);
            HIP_CHECK(hipEventRecord(gc->ev_in, stream));
            HIP_CHECK(hipStreamWaitEvent(gc->stream, gc->ev_in, 0));
        }
        hipStream_t run = use_graph ? gc->stream : stream;
        size_t k = 0;
        for (int64_t t = t0; t < t1; ++t) {
            if (ckpt && p->ckpt_every > 0 && t % p->ckpt_every == 0) {
                double* slot = ckpt + (t / p->ckpt_every) * M;
                if (identity) HIP_CHECK(hipMemcpyAsync(slot, zs, M * 8, hipMemcpyDeviceToDevice, run));
                else launch_permute_sets(zs, slot, g.N, (int32_t)nops, (int32_t)nsets, fb.perm, true, run);
            }
            if (phase_width(t) != P.nsets) {
                // the sets past the new width have finished: their columns go
                // to the caller's state, the others are repacked into the
                // other buffer, and the stage operand and Hamiltonian column
                // are remade from them (the values the last stage wrote)
                const int32_t Wo = P.nsets, W = phase_width(t);
                const double* zo = P.z;
                launch_move_sets(zo, Wo, z, (int32_t)nsets, g.N, (int32_t)nops, W, Wo, fb.perm, true, run);
                enter(++k);
                launch_move_sets(zo, Wo, P.z, W, g.N, (int32_t)nops, 0, W, nullptr, false, run);
                launch_prep_state(P.z, g.N, (int32_t)nops, W, fb.xsh[0], f32, fb.hst, run);
            }
            const int64_t c = width_class(t);
            if (use_graph) {
                hipGraphExec_t ex = nullptr;
                const int64_t id = graph_id(k, c);
                for (auto& e : gc->cls)
                    if (e.id == id) ex = e.exec;
                HIP_CHECK(hipGraphLaunch(ex, run));
            } else {
                set_class(c);
                enqueue_step(P, run, timed ? &timer : nullptr);
            }
        }
        if (zs != z) {
            launch_move_sets(P.z, P.nsets, z, (int32_t)nsets, g.N, (int32_t)nops, 0, P.nsets, fb.perm, true, run);
            if (outside)
                launch_move_sets(P.onorm, (int32_t)nsets, p->outside_norm2, (int32_t)nsets, 1, (int32_t)nops, 0,
                                 (int32_t)nsets, fb.perm, true, run);
        }
        if (timed) {
            HIP_CHECK(hipStreamSynchronize(run));
            for (size_t q = 0; q + 1 < timer.used; q += 2) {
                float ms = 0.f;
                HIP_CHECK(hipEventElapsedTime(&ms, timer.ev[q], timer.ev[q + 1]));
                if (timer.kind[q / 2] == 0) {
                    g.timing.pass_ms += ms;
                    g.timing.pass_launches++;
                } else {
                    g.timing.gen_ms += ms;
                    g.timing.gen_launches++;
                }
            }
        }
        launch_finite_check(z, M, flagp, run);
        if (use_graph) {
            HIP_CHECK(hipEventRecord(gc->ev_out, run));
            HIP_CHECK(hipStreamWaitEvent(stream, gc->ev_out, 0));
        }
        HIP_CHECK(hipGetLastError());
        if (p->nonfinite) return CUT_OK;
        int32_t flag = 0;
        HIP_CHECK(hipMemcpyAsync(&flag, fb.flag, 4, hipMemcpyDeviceToHost, stream));
        HIP_CHECK(hipStreamSynchronize(stream));
        if (flag) CUT_FAIL(CUT_E_NUMERIC, "flow produced non-finite coefficients");
        return CUT_OK;
    } catch (const Fail& f) {
        return f.st;
    } catch (const std::bad_alloc&) {
        set_error("out of host memory");
        return CUT_E_NOMEM;
    }
}

// J(Z)^T mu for f(Z) = L(eta(Z_h)) Z, all FP64:
//   u      = adjoint-x pass (j-grouped records) with eta(Z_h)
//   geta   = adjoint-eta pass (i-grouped records) of (mu, Z)
//   u_h   += eta'(Z_h)^T geta
static void jt(Graph& g, const cut_flow_params* p, int32_t nsets, int32_t nops, const double* Z, const double* mu,
               double* u, double* eta, double* geta, double* tmp, const int32_t* nsteps, const int32_t* step,
               hipStream_t s) {
    const int64_t cols = (int64_t)nops * nsets;
    eval_generator(g, p->generator, p->delta, nsets, Z, cols, eta, nsets, false, nsteps, step, s);
    PassArgs a{};
    a.nsets = nsets;
    a.nops = nops;
    a.precision = CUT_F64;
    a.nsteps = nsteps;
    a.step = step;
    a.scale = 1.0;
    a.csr = &g.csr[0][1];
    a.A = eta;
    a.lda = nsets;
    a.B = mu;
    a.ldb = cols;
    a.y = u;
    a.ldy = cols;
    launch_pass(MODE_BCAST, EPI_Y, a, s);
    a.csr = &g.csr[0][2];
    a.A = mu;
    a.lda = cols;
    a.B = Z;
    a.ldb = cols;
    a.y = geta;
    a.ldy = nsets;
    launch_pass(MODE_REDOPS, EPI_Y, a, s);
    eval_generator_vjp(g, p->generator, p->delta, nsets, Z, cols, geta, nsets, u, cols, tmp, s);
}

extern "C" cut_status cut_flow_adjoint(cut_graph_t h, const cut_flow_params* p, int64_t nsets, int64_t nops,
                                       const int32_t* n_steps, const double* ckpt, double* lambda, void* stream_) {
    try {
        Graph& g = checked(h);
        check_flow(g, p, nsets, nops, n_steps);
        if (!g.have_adjoint) CUT_FAIL(CUT_E_INVAL, "flow adjoint needs a graph loaded with CUT_LOAD_ADJOINT");
        if (!ckpt || !lambda || p->ckpt_every <= 0)
            CUT_FAIL(CUT_E_INVAL, "flow adjoint needs checkpoints (ckpt_every > 0) and lambda");
        DeviceGuard dg(g.device);
        hipStream_t s = (hipStream_t)stream_;
        int64_t T = 0;
        for (int64_t q = 0; q < nsets; ++q) T = std::max<int64_t>(T, n_steps[q]);
        if (T == 0) return CUT_OK;
        const int64_t cols = nops * nsets, M = g.N * cols;
        const int C = p->ckpt_every;
        const int64_t nslot = (int64_t)C * 4 + 1;
        const size_t extra = flow_adjoint_extra(g, nsets, nops, C);
        char* ex = nullptr;
        FlowBufs fb = flow_bufs(g, nsets, nops, CUT_F64, extra, &ex);
        double* St = (double*)ex;
        ex += al(nslot * M * 8);
        double* zr = (double*)ex;
        ex += al(M * 8);
        double* lam_new = (double*)ex;
        ex += al(M * 8);
        double* mu = (double*)ex;
        ex += al(M * 8);
        double* u = (double*)ex;
        ex += al(M * 8);
        double* eta = (double*)ex;
        ex += al(g.NG * nsets * 8);
        double* geta = (double*)ex;
        ex += al(g.NG * nsets * 8);
        double* tmp = (double*)ex;
        HIP_CHECK(hipMemcpyAsync(fb.nsteps, n_steps, nsets * 4, hipMemcpyHostToDevice, s));
        const int64_t nblk = (T + C - 1) / C;
        const double ds = p->ds;
        for (int64_t b = nblk - 1; b >= 0; --b) {
            const int64_t t0 = b * C, t1 = std::min<int64_t>(T, t0 + C);
            // recompute the block forward in FP64, keeping every stage state:
            // stage st of local step l reads St[4l+st] and writes St[4l+st+1]
            HIP_CHECK(hipMemcpyAsync(zr, ckpt + b * M, M * 8, hipMemcpyDeviceToDevice, s));
            launch_prep_state(zr, g.N, (int32_t)nops, (int32_t)nsets, St, false, fb.hst, s);
            launch_set_scalar(fb.step, (int32_t)t0, s);
            StepPlan P{&g, p->generator, CUT_F64, ds, p->delta, (int32_t)nsets, (int32_t)nops, fb, zr, {}, {}};
            for (int64_t t = t0; t < t1; ++t) {
                const int64_t l = t - t0;
                for (int st = 0; st < 4; ++st) {
                    P.xin[st] = St + (4 * l + st) * M;
                    P.xout[st] = St + (4 * l + st + 1) * M;
                }
                enqueue_step(P, s);
            }
            for (int64_t t = t1 - 1; t >= t0; --t) {
                const int64_t l = t - t0;
                launch_set_scalar(fb.step, (int32_t)t, s);
                const double* Zs[4] = {St + (4 * l) * M, St + (4 * l + 1) * M, St + (4 * l + 2) * M,
                                       St + (4 * l + 3) * M};
                // u4 = J(Z4)^T [ds/6 lam]
                launch_adj_combine(g.N, (int32_t)cols, (int32_t)nsets, fb.nsteps, fb.step, lambda, nullptr, lam_new,
                                   mu, ds / 6.0, 0.0, 1, s);
                jt(g, p, (int32_t)nsets, (int32_t)nops, Zs[3], mu, u, eta, geta, tmp, fb.nsteps, fb.step, s);
                launch_adj_combine(g.N, (int32_t)cols, (int32_t)nsets, fb.nsteps, fb.step, lambda, u, lam_new, mu,
                                   ds / 3.0, ds, 0, s);
                jt(g, p, (int32_t)nsets, (int32_t)nops, Zs[2], mu, u, eta, geta, tmp, fb.nsteps, fb.step, s);
                launch_adj_combine(g.N, (int32_t)cols, (int32_t)nsets, fb.nsteps, fb.step, lambda, u, lam_new, mu,
                                   ds / 3.0, 0.5 * ds, 0, s);
                jt(g, p, (int32_t)nsets, (int32_t)nops, Zs[1], mu, u, eta, geta, tmp, fb.nsteps, fb.step, s);
                launch_adj_combine(g.N, (int32_t)cols, (int32_t)nsets, fb.nsteps, fb.step, lambda, u, lam_new, mu,
                                   ds / 6.0, 0.5 * ds, 0, s);
                jt(g, p, (int32_t)nsets, (int32_t)nops, Zs[0], mu, u, eta, geta, tmp, fb.nsteps, fb.step, s);
                launch_adj_combine(g.N, (int32_t)cols, (int32_t)nsets, fb.nsteps, fb.step, lambda, u, lam_new,
                                   nullptr, 0.0, 0.0, 0, s);
                launch_copy_active(g.N, (int32_t)cols, (int32_t)nsets, fb.nsteps, fb.step, lam_new, lambda, s);
            }
        }
        int32_t* const flagp = p->nonfinite ? p->nonfinite : fb.flag;
        launch_set_scalar(flagp, 0, s);
        launch_finite_check(lambda, M, flagp, s);
        HIP_CHECK(hipGetLastError());
        if (p->nonfinite) return CUT_OK;
        int32_t flag = 0;
        HIP_CHECK(hipMemcpyAsync(&flag, fb.flag, 4, hipMemcpyDeviceToHost, s));
        HIP_CHECK(hipStreamSynchronize(s));
        if (flag) CUT_FAIL(CUT_E_NUMERIC, "adjoint produced non-finite values");
        return CUT_OK;
    } catch (const Fail& f) {
        return f.st;
    } catch (const std::bad_alloc&) {
        set_error("out of host memory");
        return CUT_E_NOMEM;
    }
}

extern "C" cut_status cut_flow_last_timing(cut_graph_t h, cut_flow_timing* t) {
    if (!h || !t) {
        set_error("cut_flow_last_timing: null argument");
        return CUT_E_INVAL;
    }
    *t = ((Graph*)h)->timing;
    return CUT_OK;
}
