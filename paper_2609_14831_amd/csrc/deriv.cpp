// Derivatives of one projected action F(h, x) = L(eta(h)) x (Sec. 2.4):
// the directional derivative of Eq. directional-derivative (the induced
// generator variation plus the linear response to the operand) and its
// transpose (the adjoint traversals of the same records followed by the
// generator VJP).  Both are sequences of the generator kernels and graph
// passes; nothing here forms a Jacobian.
#include <vector>

#include "internal.h"

namespace cut {

// deta[N][nsets] = eta'(h) dh  (FP64)
void eval_generator_jvp(Graph& g, int kind, double delta, int32_t nsets, const double* h, int64_t ldh,
                        const double* dh, int64_t lddh, double* deta, int64_t ldde, hipStream_t s) {
    if (kind == CUT_GEN_G2) {
        launch_g2_jvp(g, delta, nsets, h, ldh, dh, lddh, deta, ldde, s);
        return;
    }
    if (kind == CUT_GEN_G1) {
        launch_g1_jvp(g, delta, nsets, h, ldh, dh, lddh, deta, ldde, s);
        return;
    }
    // eta_k = s_g sum_{E_eta(k)} c h_i h_j with i block-diagonal and j not (the
    // only records with a nonzero bracket), so by the product rule
    // deta_k = s_g sum c (dh_i h_j + h_i dh_j): two passes over the same records
    PassArgs p{};
    p.csr = &g.csr[1][0];
    p.nsets = nsets;
    p.nops = 1;
    p.precision = CUT_F64;
    p.y = deta;
    p.ldy = ldde;
    p.scale = g.gen_sign;
    p.A = dh;
    p.lda = lddh;
    p.B = h;
    p.ldb = ldh;
    p.accumulate = 0;
    launch_pass(MODE_BCAST, EPI_Y, p, s);
    p.A = h;
    p.lda = ldh;
    p.B = dh;
    p.ldb = lddh;
    p.accumulate = 1;
    launch_pass(MODE_BCAST, EPI_Y, p, s);
}

namespace {

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

// Bump allocator over the derivative work area: sizes are summed first, the
// area is grown once, then the pointers are handed out in the same order.
struct Carve {
    size_t total = 0;
    std::vector<size_t> offs;
    size_t add(size_t bytes) {
        offs.push_back(total);
        total += al(bytes);
        return offs.size() - 1;
    }
};

// work area of cut_graph_jvp: eta, deta (FP64), their float shadows, float x / dx
struct JvpLayout {
    Carve cv;
    size_t eta, deta, deta32, x32, dx32;
    JvpLayout(const Graph& g, int64_t nsets, int64_t nops, int precision, bool dh, bool dx, bool need_x) {
        const bool f32 = precision != CUT_F64;
        const size_t tb = f32 ? 4 : 8;
        const int64_t N = g.N, NG = g.NG, cols = nops * nsets;
        eta = cv.add(NG * nsets * tb);
        deta = cv.add(dh ? NG * nsets * 8 : 0);
        deta32 = cv.add(dh && f32 ? NG * nsets * 4 : 0);
        x32 = cv.add(need_x && f32 ? N * cols * 4 : 0);
        dx32 = cv.add(dx && f32 ? N * cols * 4 : 0);
    }
};

// work area of cut_graph_vjp: eta, float w / x, geta, generator-VJP scratch
struct VjpLayout {
    Carve cv;
    size_t eta, w32, x32, geta, tmp;
    VjpLayout(const Graph& g, int64_t nsets, int64_t nops, int precision, bool gx, bool gh, bool g2) {
        const bool f32 = precision != CUT_F64;
        const int64_t N = g.N, NG = g.NG, cols = nops * nsets;
        eta = cv.add(gx ? NG * nsets * (f32 ? 4 : 8) : 0);
        w32 = cv.add(f32 ? N * cols * 4 : 0);
        x32 = cv.add(gh && f32 ? N * cols * 4 : 0);
        geta = cv.add(gh ? NG * nsets * 8 : 0);
        tmp = cv.add(gh && g2 ? 2 * N * nsets * 8 : 0);
    }
};

}  // namespace

size_t jvp_ws_bytes(const Graph& g, int64_t nsets, int64_t nops, int prec) {
    return JvpLayout(g, nsets, nops, prec, true, true, true).cv.total;
}

size_t vjp_ws_bytes(const Graph& g, int64_t nsets, int64_t nops, int prec) {
    return VjpLayout(g, nsets, nops, prec, true, true, true).cv.total;
}

}  // namespace cut

using namespace cut;

extern "C" cut_status cut_generator_jvp(cut_graph_t hd, int32_t kind, double delta, int64_t nsets,
                                        const double* h, int64_t ldh, const double* dh, int64_t lddh,
                                        double* deta, int64_t ldde, void* stream) {
    ABI_BEGIN
    Graph& g = checked(hd);
    check_generator(g, kind);
    check_shape(nsets, 1);
    if (!h || !dh || !deta || ldh < nsets || lddh < nsets || ldde < nsets)
        CUT_FAIL(CUT_E_INVAL, "cut_generator_jvp: bad operand");
    DeviceGuard dg(g.device);
    eval_generator_jvp(g, kind, delta, (int32_t)nsets, h, ldh, dh, lddh, deta, ldde, (hipStream_t)stream);
    HIP_CHECK(hipGetLastError());
    ABI_END
}

extern "C" cut_status cut_graph_jvp(cut_graph_t hd, int32_t kind, double delta, int32_t precision, int64_t nsets,
                                    int64_t nops, const double* h, int64_t ldh, const double* dh, int64_t lddh,
                                    const double* x, int64_t ldx, const double* dx, int64_t lddx, double* y,
                                    int64_t ldy, double* dy, int64_t lddy, void* stream) {
    ABI_BEGIN
    Graph& g = checked(hd);
    check_generator(g, kind);
    check_prec(precision);
    check_shape(nsets, nops);
    const int64_t cols = nops * nsets;
    if (!h || ldh < nsets) CUT_FAIL(CUT_E_INVAL, "cut_graph_jvp: bad h");
    if (!dy || lddy < cols) CUT_FAIL(CUT_E_INVAL, "cut_graph_jvp: bad dy");
    if (!dh && !dx) CUT_FAIL(CUT_E_INVAL, "cut_graph_jvp: both tangents are NULL");
    if (dh && lddh < nsets) CUT_FAIL(CUT_E_INVAL, "cut_graph_jvp: bad dh");
    if (dx && lddx < cols) CUT_FAIL(CUT_E_INVAL, "cut_graph_jvp: bad dx");
    if ((dh || y) && (!x || ldx < cols)) CUT_FAIL(CUT_E_INVAL, "cut_graph_jvp: bad x");
    if (y && ldy < cols) CUT_FAIL(CUT_E_INVAL, "cut_graph_jvp: bad y");
    DeviceGuard dg(g.device);
    hipStream_t s = (hipStream_t)stream;
    const bool f32 = precision != CUT_F64;
    const size_t tb = f32 ? 4 : 8;
    const int64_t N = g.N;
    const bool need_x = dh || y;
    const JvpLayout lay(g, nsets, nops, precision, dh != nullptr, dx != nullptr, need_x);
    const Carve& cv = lay.cv;
    const int64_t NG = g.NG;
    const size_t i_eta = lay.eta, i_deta = lay.deta, i_deta32 = lay.deta32, i_x32 = lay.x32, i_dx32 = lay.dx32;
    char* base = (char*)g.ws_deriv.need(cv.total, "cut_graph_jvp");
    auto at = [&](size_t i) { return (void*)(base + cv.offs[i]); };
    const size_t pb = forward_partial_bytes(g, (int32_t)nsets, (int32_t)nops, precision);
    double* part = pb ? (double*)g.ws_part.need(pb, "cut_graph_jvp (partial rows)") : nullptr;

    // eta(h) in the pass precision (rounded once for the float modes)
    void* eta = at(i_eta);
    eval_generator(g, kind, delta, (int32_t)nsets, h, ldh, eta, nsets, f32, nullptr, nullptr, s);
    // deta = eta'(h) dh in FP64, then its float shadow
    const void* deta = nullptr;
    if (dh) {
        double* d64 = (double*)at(i_deta);
        eval_generator_jvp(g, kind, delta, (int32_t)nsets, h, ldh, dh, lddh, d64, nsets, s);
        deta = d64;
        if (f32) {
            launch_round_f32(d64, nsets, NG, nsets, (float*)at(i_deta32), nsets, s);
            deta = at(i_deta32);
        }
    }
    const void* xo = x;
    int64_t ldxo = ldx;
    if (need_x && f32) {
        launch_round_f32(x, ldx, N, cols, (float*)at(i_x32), cols, s);
        xo = at(i_x32);
        ldxo = cols;
    }
    const void* dxo = dx;
    int64_t lddxo = lddx;
    if (dx && f32) {
        launch_round_f32(dx, lddx, N, cols, (float*)at(i_dx32), cols, s);
        dxo = at(i_dx32);
        lddxo = cols;
    }

    PassArgs p{};
    p.csr = &g.csr[0][0];
    p.nsets = (int32_t)nsets;
    p.nops = (int32_t)nops;
    p.precision = precision;
    p.scale = 1.0;
    p.lda = nsets;
    // dy = apply(deta, x) + apply(eta, dx)
    p.y = dy;
    p.ldy = lddy;
    p.accumulate = 0;
    if (dh) {
        p.A = deta;
        p.B = xo;
        p.ldb = ldxo;
        launch_forward(g, EPI_Y, p, part, s);
        p.accumulate = 1;
    }
    if (dx) {
        p.A = eta;
        p.B = dxo;
        p.ldb = lddxo;
        launch_forward(g, EPI_Y, p, part, s);
    }
    // y = apply(eta, x)
    if (y) {
        p.A = eta;
        p.B = xo;
        p.ldb = ldxo;
        p.y = y;
        p.ldy = ldy;
        p.accumulate = 0;
        launch_forward(g, EPI_Y, p, part, s);
    }
    HIP_CHECK(hipGetLastError());
    ABI_END
}

extern "C" cut_status cut_graph_vjp(cut_graph_t hd, int32_t kind, double delta, int32_t precision, int64_t nsets,
                                    int64_t nops, const double* h, int64_t ldh, const double* x, int64_t ldx,
                                    const double* w, int64_t ldw, double* g_h, int64_t ldgh, double* g_x,
                                    int64_t ldgx, uint32_t flags, void* stream) {
    ABI_BEGIN
    Graph& g = checked(hd);
    check_generator(g, kind);
    check_prec(precision);
    check_shape(nsets, nops);
    if (!g.have_adjoint) CUT_FAIL(CUT_E_INVAL, "cut_graph_vjp needs a graph loaded with CUT_LOAD_ADJOINT");
    const int64_t cols = nops * nsets;
    if (!h || ldh < nsets) CUT_FAIL(CUT_E_INVAL, "cut_graph_vjp: bad h");
    if (!w || ldw < cols) CUT_FAIL(CUT_E_INVAL, "cut_graph_vjp: bad w");
    if (!g_h && !g_x) CUT_FAIL(CUT_E_INVAL, "cut_graph_vjp: both outputs are NULL");
    if (g_h && (ldgh < nsets || !x || ldx < cols)) CUT_FAIL(CUT_E_INVAL, "cut_graph_vjp: bad g_h / x");
    if (g_x && ldgx < cols) CUT_FAIL(CUT_E_INVAL, "cut_graph_vjp: bad g_x");
    DeviceGuard dg(g.device);
    hipStream_t s = (hipStream_t)stream;
    const bool f32 = precision != CUT_F64;
    const bool acc = (flags & CUT_ACCUMULATE) != 0;
    const int64_t N = g.N;
    const VjpLayout lay(g, nsets, nops, precision, g_x != nullptr, g_h != nullptr, stencil_generator(kind));
    const Carve& cv = lay.cv;
    const int64_t NG = g.NG;
    const size_t i_eta = lay.eta, i_w32 = lay.w32, i_x32 = lay.x32, i_geta = lay.geta, i_tmp = lay.tmp;
    char* base = (char*)g.ws_deriv.need(cv.total, "cut_graph_vjp");
    auto at = [&](size_t i) { return (void*)(base + cv.offs[i]); };

    const void* wo = w;
    int64_t ldwo = ldw;
    if (f32) {
        launch_round_f32(w, ldw, N, cols, (float*)at(i_w32), cols, s);
        wo = at(i_w32);
        ldwo = cols;
    }
    PassArgs p{};
    p.nsets = (int32_t)nsets;
    p.nops = (int32_t)nops;
    p.precision = precision;
    p.scale = 1.0;
    if (g_x) {
        // g_x (=|+=) L(eta)^T w: the record copy grouped by right input j
        void* eta = at(i_eta);
        eval_generator(g, kind, delta, (int32_t)nsets, h, ldh, eta, nsets, f32, nullptr, nullptr, s);
        p.csr = &g.csr[0][1];
        p.A = eta;
        p.lda = nsets;
        p.B = wo;
        p.ldb = ldwo;
        p.y = g_x;
        p.ldy = ldgx;
        p.accumulate = acc ? 1 : 0;
        launch_pass(MODE_BCAST, EPI_Y, p, s);
    }
    if (g_h) {
        // geta = sum over the records grouped by left input i of c sum_op w_k x_j,
        // then g_h (=|+=) eta'(h)^T geta
        const void* xo = x;
        int64_t ldxo = ldx;
        if (f32) {
            launch_round_f32(x, ldx, N, cols, (float*)at(i_x32), cols, s);
            xo = at(i_x32);
            ldxo = cols;
        }
        double* geta = (double*)at(i_geta);
        p.csr = &g.csr[0][2];
        p.A = wo;
        p.lda = ldwo;
        p.B = xo;
        p.ldb = ldxo;
        p.y = geta;
        p.ldy = nsets;
        p.accumulate = 0;
        launch_pass(MODE_REDOPS, EPI_Y, p, s);
        if (!acc) launch_zero2d(g_h, ldgh, N, nsets, s);
        eval_generator_vjp(g, kind, delta, (int32_t)nsets, h, ldh, geta, nsets, g_h, ldgh,
                           stencil_generator(kind) ? (double*)at(i_tmp) : nullptr, s);
    }
    HIP_CHECK(hipGetLastError());
    ABI_END
}
