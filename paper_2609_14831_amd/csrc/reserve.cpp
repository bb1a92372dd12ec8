// Work-area reservation.  The computing entry points (actions, derivatives,
// flows) never allocate or synchronise: they carve their scratch out of work
// areas that only cut_graph_reserve and the tiling calls size.
#include <algorithm>

#include "internal.h"

namespace cut {

void reserve_shape(Graph& g, int64_t nsets, int64_t nops, int64_t ckpt_every, uint32_t what) {
    size_t part = 0, small = 0, deriv = 0, ws = 0;
    for (int prec = CUT_F64; prec <= CUT_F32; ++prec) {
        if (what & (CUT_RESERVE_APPLY | CUT_RESERVE_DERIV))
            part = std::max(part, forward_partial_bytes(g, (int32_t)nsets, (int32_t)nops, prec));
        if (what & CUT_RESERVE_DERIV)
            deriv = std::max({deriv, jvp_ws_bytes(g, nsets, nops, prec), vjp_ws_bytes(g, nsets, nops, prec)});
        if (what & CUT_RESERVE_FLOW)
            ws = std::max(ws, flow_ws_bytes(g, nsets, nops, prec, flow_outside_extra(g, nsets, nops)));
    }
    if (what & CUT_RESERVE_APPLY) small = sizeof(double) * 2 * g.N * nsets;
    if ((what & CUT_RESERVE_ADJOINT) && ckpt_every > 0)
        ws = std::max(ws, flow_ws_bytes(g, nsets, nops, CUT_F64, flow_adjoint_extra(g, nsets, nops, ckpt_every)));
    g.ws_part.reserve(part);
    g.ws_small.reserve(small);
    g.ws_deriv.reserve(deriv);
    g.ws.reserve(ws);
}

void rereserve(Graph& g) {
    for (const auto& r : g.reserved) reserve_shape(g, r[0], r[1], r[2], (uint32_t)r[3]);
}

}  // namespace cut

using namespace cut;

extern "C" cut_status cut_graph_reserve(cut_graph_t h, int64_t nsets, int64_t nops, int64_t ckpt_every,
                                        uint32_t what) {
    ABI_BEGIN
    Graph& g = checked(h);
    check_shape(nsets, nops);
    if (what == 0 || (what & ~15u)) CUT_FAIL(CUT_E_INVAL, "cut_graph_reserve: unknown flags 0x%x", what);
    if (ckpt_every < 0 || ((what & CUT_RESERVE_ADJOINT) && ckpt_every == 0))
        CUT_FAIL(CUT_E_INVAL, "cut_graph_reserve: CUT_RESERVE_ADJOINT needs ckpt_every > 0");
    DeviceGuard dg(g.device);
    reserve_shape(g, nsets, nops, ckpt_every, what);
    const std::vector<int64_t> key = {nsets, nops, ckpt_every, (int64_t)what};
    if (std::find(g.reserved.begin(), g.reserved.end(), key) == g.reserved.end()) g.reserved.push_back(key);
    ABI_END
}

extern "C" cut_status cut_graph_reserved_bytes(cut_graph_t h, int64_t* bytes) {
    ABI_BEGIN
    Graph& g = checked(h);
    if (!bytes) CUT_FAIL(CUT_E_INVAL, "cut_graph_reserved_bytes: null output");
    *bytes = (int64_t)(g.ws.bytes + g.ws_small.bytes + g.ws_part.bytes + g.ws_deriv.bytes);
    ABI_END
}
