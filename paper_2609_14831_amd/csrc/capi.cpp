// C ABI: single graph actions (Sec. 2.2 Eq. graph-actions; Sec. 2.4 adjoint)
// and generator evaluation (Sec. 2.1 Eq. block-generator).
#include <cstring>

#include "internal.h"

namespace cut {

DeviceGuard::DeviceGuard(int dev) {
    HIP_CHECK(hipGetDevice(&prev));
    if (prev != dev) HIP_CHECK(hipSetDevice(dev));
}
DeviceGuard::~DeviceGuard() {
    int cur = -1;
    if (hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
}

Graph& checked(cut_graph_t h) {
    if (!h) CUT_FAIL(CUT_E_INVAL, "null graph handle");
    return *(Graph*)h;
}

void check_prec(int p) {
    if (p < CUT_F64 || p > CUT_F32) CUT_FAIL(CUT_E_INVAL, "unknown precision %d", p);
}

void check_shape(int64_t nsets, int64_t nops) {
    if (nsets < 1 || nsets > (1 << 20)) CUT_FAIL(CUT_E_INVAL, "nsets %lld out of range", (long long)nsets);
    if (nops < 1 || nops > 8) CUT_FAIL(CUT_E_INVAL, "nops %lld outside 1..8", (long long)nops);
}

bool gen_graph_ok(const Graph& g) {
    return g.csr[1][0].nseg > 0 || g.hdr.n_gen_records == 0;
}

// eta[N][nsets] (ld lde, double or float) from h (double, ld ldh)
void eval_generator(Graph& g, int kind, double delta, int32_t nsets, const double* h, int64_t ldh, void* eta,
                    int64_t lde, bool eta_f32, const int32_t* nsteps, const int32_t* step, hipStream_t s) {
    if (kind == CUT_GEN_G2) {
        launch_g2(g, delta, nsets, h, ldh, eta, lde, eta_f32, nsteps, step, s);
    } else if (kind == CUT_GEN_G1) {
        launch_g1(g, delta, nsets, h, ldh, eta, lde, eta_f32, nsteps, step, s);
    } else {
        PassArgs p{};
        p.csr = &g.csr[1][0];
        p.A = h;
        p.lda = ldh;
        p.B = h;
        p.ldb = ldh;
        p.nsets = nsets;
        p.nops = 1;
        p.precision = eta_f32 ? CUT_F32X : CUT_F64;
        p.nsteps = nsteps;
        p.step = step;
        p.y = eta;
        p.ldy = lde;
        p.scale = g.gen_sign;
        launch_pass(MODE_BCAST, EPI_ETA, p, s);
    }
}

void check_generator(const Graph& g, int kind) {
    if (stencil_generator(kind)) {
        if (g.hdr.algebra != CUT_ALG_MAJORANA || !g.have_stencil)
            CUT_FAIL(CUT_E_UNSUPPORTED, "G1 / G2 generators need a pair-flip registry (Majorana strings)");
    } else if (kind != CUT_GEN_WEGNER_GRAPH) {
        CUT_FAIL(CUT_E_INVAL, "unknown generator %d", kind);
    }
}

// g_h[N][nsets] += eta'(h)^T gbar
// tmp: 2*N*nsets doubles of scratch (G2 only)
void eval_generator_vjp(Graph& g, int kind, double delta, int32_t nsets, const double* h, int64_t ldh,
                        const double* gbar, int64_t ldg, double* g_h, int64_t ldgh, double* tmp,
                        hipStream_t s) {
    if (kind == CUT_GEN_G2) {
        launch_g2_vjp(g, delta, nsets, h, ldh, gbar, ldg, g_h, ldgh, tmp, s);
        return;
    }
    if (kind == CUT_GEN_G1) {
        launch_g1_vjp(g, delta, nsets, h, ldh, gbar, ldg, g_h, ldgh, tmp, s);
        return;
    }
    if (!g.have_adjoint) CUT_FAIL(CUT_E_INVAL, "generator VJP needs a graph loaded with CUT_LOAD_ADJOINT");
    // eta_k = s_g sum c h_i h_j over E_eta: d/dh_i via the i-grouped copy,
    // d/dh_j via the j-grouped copy, both accumulated into g_h
    PassArgs p{};
    p.nsets = nsets;
    p.nops = 1;
    p.precision = CUT_F64;
    p.y = g_h;
    p.ldy = ldgh;
    p.accumulate = 1;
    p.scale = g.gen_sign;
    p.csr = &g.csr[1][2];  // by i: a = k, b = j
    p.A = gbar;
    p.lda = ldg;
    p.B = h;
    p.ldb = ldh;
    launch_pass(MODE_BCAST, EPI_Y, p, s);
    p.csr = &g.csr[1][1];  // by j: a = i, b = k
    p.A = h;
    p.lda = ldh;
    p.B = gbar;
    p.ldb = ldg;
    launch_pass(MODE_BCAST, EPI_Y, p, s);
}

}  // namespace cut

using namespace cut;

namespace cut {

// Validates the arguments of a forward action and returns its pass arguments;
// *part_bytes receives the partial-row bytes its forward pass needs (0: none).
PassArgs apply_args(Graph& g, int32_t which, int32_t precision, int64_t nsets, int64_t nops, const void* eta,
                    int64_t lde, const void* x, int64_t ldx, double* y, int64_t ldy, uint32_t flags,
                    size_t* part_bytes) {
    if (which != CUT_GRAPH_FLOW && which != CUT_GRAPH_GEN && which != CUT_GRAPH_OUTSIDE)
        CUT_FAIL(CUT_E_INVAL, "unknown record set %d", which);
    if (which == CUT_GRAPH_OUTSIDE && !g.have_outside)
        CUT_FAIL(CUT_E_INVAL, "cut_graph_apply: the bundle has no outside-space records");
    check_prec(precision);
    check_shape(nsets, nops);
    if (!eta || !x || !y) CUT_FAIL(CUT_E_INVAL, "cut_graph_apply: null operand");
    if (lde < nsets || ldx < nops * nsets || ldy < nops * nsets)
        CUT_FAIL(CUT_E_INVAL, "cut_graph_apply: leading dimension too small");
    PassArgs p{};
    p.csr = &g.csr[which][0];
    p.A = eta;
    p.lda = lde;
    p.B = x;
    p.ldb = ldx;
    p.nsets = (int32_t)nsets;
    p.nops = (int32_t)nops;
    p.precision = precision;
    p.y = y;
    p.ldy = ldy;
    p.accumulate = (flags & CUT_ACCUMULATE) ? 1 : 0;
    p.scale = 1.0;
    *part_bytes = which == CUT_GRAPH_FLOW ? forward_partial_bytes(g, p.nsets, p.nops, precision) : 0;
    return p;
}

}  // namespace cut

extern "C" cut_status cut_graph_apply(cut_graph_t h, int32_t which, int32_t precision, int64_t nsets,
                                      int64_t nops, const void* eta, int64_t lde, const void* x, int64_t ldx,
                                      double* y, int64_t ldy, uint32_t flags, void* stream) {
    ABI_BEGIN
    Graph& g = checked(h);
    size_t pb = 0;
    const PassArgs p = apply_args(g, which, precision, nsets, nops, eta, lde, x, ldx, y, ldy, flags, &pb);
    DeviceGuard dg(g.device);
    double* part = pb ? (double*)g.ws_part.need(pb, "cut_graph_apply (partial rows)") : nullptr;
    launch_forward(g, EPI_Y, p, part, (hipStream_t)stream);
    HIP_CHECK(hipGetLastError());
    ABI_END
}

extern "C" cut_status cut_graph_apply_adjoint(cut_graph_t h, int32_t which, int32_t precision, int64_t nsets,
                                              int64_t nops, const void* eta, int64_t lde, const void* x,
                                              int64_t ldx, const void* w, int64_t ldw, double* g_x, int64_t ldgx,
                                              double* g_eta, int64_t ldge, uint32_t flags, void* stream) {
    ABI_BEGIN
    Graph& g = checked(h);
    if (which != CUT_GRAPH_FLOW && which != CUT_GRAPH_GEN)
        CUT_FAIL(CUT_E_INVAL, "cut_graph_apply_adjoint: record set %d has no adjoint copies", which);
    check_prec(precision);
    check_shape(nsets, nops);
    if (!g.have_adjoint) CUT_FAIL(CUT_E_INVAL, "adjoint needs a graph loaded with CUT_LOAD_ADJOINT");
    if (!w || ldw < nops * nsets) CUT_FAIL(CUT_E_INVAL, "cut_graph_apply_adjoint: bad w");
    if (g_x && (!eta || lde < nsets || ldgx < nops * nsets))
        CUT_FAIL(CUT_E_INVAL, "cut_graph_apply_adjoint: bad eta / g_x");
    if (g_eta && (!x || ldx < nops * nsets || ldge < nsets))
        CUT_FAIL(CUT_E_INVAL, "cut_graph_apply_adjoint: bad x / g_eta");
    DeviceGuard dg(g.device);
    PassArgs p{};
    p.nsets = (int32_t)nsets;
    p.nops = (int32_t)nops;
    p.precision = precision;
    p.accumulate = (flags & CUT_ACCUMULATE) ? 1 : 0;
    p.scale = 1.0;
    if (g_x) {
        p.csr = &g.csr[which][1];  // by j: a = i, b = k
        p.A = eta;
        p.lda = lde;
        p.B = w;
        p.ldb = ldw;
        p.y = g_x;
        p.ldy = ldgx;
        launch_pass(MODE_BCAST, EPI_Y, p, (hipStream_t)stream);
    }
    if (g_eta) {
        p.csr = &g.csr[which][2];  // by i: a = k, b = j
        p.A = w;
        p.lda = ldw;
        p.B = x;
        p.ldb = ldx;
        p.y = g_eta;
        p.ldy = ldge;
        launch_pass(MODE_REDOPS, EPI_Y, p, (hipStream_t)stream);
    }
    HIP_CHECK(hipGetLastError());
    ABI_END
}

extern "C" cut_status cut_generator(cut_graph_t h, int32_t kind, double delta, int64_t nsets, const double* hh,
                                    int64_t ldh, double* eta, int64_t lde, void* stream) {
    ABI_BEGIN
    Graph& g = checked(h);
    check_generator(g, kind);
    check_shape(nsets, 1);
    if (!hh || !eta || ldh < nsets || lde < nsets) CUT_FAIL(CUT_E_INVAL, "cut_generator: bad operand");
    DeviceGuard dg(g.device);
    eval_generator(g, kind, delta, (int32_t)nsets, hh, ldh, eta, lde, false, nullptr, nullptr, (hipStream_t)stream);
    HIP_CHECK(hipGetLastError());
    ABI_END
}

extern "C" cut_status cut_generator_vjp(cut_graph_t h, int32_t kind, double delta, int64_t nsets,
                                        const double* hh, int64_t ldh, const double* gbar, int64_t ldg,
                                        double* g_h, int64_t ldgh, void* stream) {
    ABI_BEGIN
    Graph& g = checked(h);
    check_generator(g, kind);
    check_shape(nsets, 1);
    if (!hh || !gbar || !g_h || ldh < nsets || ldg < nsets || ldgh < nsets)
        CUT_FAIL(CUT_E_INVAL, "cut_generator_vjp: bad operand");
    DeviceGuard dg(g.device);
    double* tmp = stencil_generator(kind) ? (double*)g.ws_small.need(sizeof(double) * 2 * g.N * nsets, "cut_generator_vjp")
                                     : nullptr;
    eval_generator_vjp(g, kind, delta, (int32_t)nsets, hh, ldh, gbar, ldg, g_h, ldgh, tmp, (hipStream_t)stream);
    HIP_CHECK(hipGetLastError());
    ABI_END
}
