// Multi-operator assembly (Sec. 2.4, last paragraph; Sec. 3.4): output
// operators as linear combinations of a transformed source library,
//   Y[n][k] (=|+=) sum_s X[n][s] W[s][k],
// a dense FP64 product on the matrix cores (v_mfma_f64_16x16x4f64).
//
// Tiling: a workgroup of 4 wavefronts owns a 128 x 128 block of Y; wavefront w
// owns the 64 x 64 quarter (w / 2, w % 2) as 4 x 4 MFMA tiles of 16 x 16.  The
// source dimension is walked in chunks of 8: the 128 x 8 slice of X (k-major)
// and the 8 x 128 slice of W are staged in LDS (zero-filled past the edges),
// and every wavefront issues 2 k-steps x 16 tiles of MFMA per chunk.  The next
// chunk's global loads are issued before the current chunk's MFMAs and stored
// to the other of two LDS buffers after them (one barrier per chunk).  Interior
// blocks take unchecked vector loads and stores; the output is written with
// non-temporal stores.
//
// MFMA 16x16x4 FP64 operand layout (per lane l of the wavefront): A element
// (row l % 16, k = l / 16), B element (k = l / 16, column l % 16); element r of
// the result (r = 0..3) is row l / 16 + 4 r of column l % 16 (rows interleaved
// across the four lane groups; checked on the device against the oracle).
#include "internal.h"

namespace cut {
namespace {

typedef double double4_t __attribute__((ext_vector_type(4)));

// BM x BN block of Y per workgroup of 4 wavefronts (2 x 2), each wavefront a
// (BM/2) x (BN/2) quarter as TI x TJ MFMA tiles of 16 x 16; sources in chunks
// of BK staged in LDS.
template <int BM, int BN, int BK, bool ACC>
__global__ __launch_bounds__(256) void k_assemble(const double* __restrict__ X, int64_t ldx, int64_t N, int64_t S,
                                                  const double* __restrict__ W, int64_t ldw, int64_t K,
                                                  double* __restrict__ Y, int64_t ldy) {
    constexpr int TI = BM / 32, TJ = BN / 32;
    constexpr int XPT = BM * BK / 256, WPT = BK * BN / 256;   // staged elements per thread
    static_assert(BK % 4 == 0 && XPT >= 1 && WPT >= 1, "tile shape");
    // two buffers of the X slice (k-major: a fragment reads 16 consecutive
    // rows) and of the W slice, unpadded: 32 KB per workgroup
    __shared__ double xs[2][BK][BM];
    __shared__ double ws[2][BK][BN];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int64_t row0 = (int64_t)blockIdx.x * BM, col0 = (int64_t)blockIdx.y * BN;
    const int wr = (wave >> 1) * (BM / 2), wc = (wave & 1) * (BN / 2);
    // staging: thread t holds XPT consecutive k of one X row and WPT
    // consecutive columns of one W row
    constexpr int XTPR = BK / XPT;                 // threads per X row
    constexpr int WTPR = BN / WPT;                 // threads per W row
    const int xr = t / XTPR, xk = (t % XTPR) * XPT;
    const int wk = t / WTPR, wcol = (t % WTPR) * WPT;
    double xv[XPT], wv[WPT];
    // interior blocks (every row and column in range) skip the per-element
    // checks of the staging loads, and of the stores below
    const bool full = row0 + BM <= N && col0 + BN <= K;
    auto fetch = [&](int64_t k0) {
        const int64_t gr = row0 + xr;
        const int64_t gk = k0 + wk;
        if (full && k0 + BK <= S) {
            const double* xp = X + gr * ldx + k0 + xk;
            const double* wp = W + gk * ldw + col0 + wcol;
#pragma unroll
            for (int e = 0; e < XPT; ++e) xv[e] = xp[e];
#pragma unroll
            for (int e = 0; e < WPT; ++e) wv[e] = wp[e];
            return;
        }
#pragma unroll
        for (int e = 0; e < XPT; ++e) {
            const int64_t k = k0 + xk + e;
            xv[e] = (gr < N && k < S) ? X[gr * ldx + k] : 0.0;
        }
#pragma unroll
        for (int e = 0; e < WPT; ++e) {
            const int64_t gc = col0 + wcol + e;
            wv[e] = (gk < S && gc < K) ? W[gk * ldw + gc] : 0.0;
        }
    };
    double4_t acc[TI][TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) acc[i][j] = double4_t{0.0, 0.0, 0.0, 0.0};

    // chunk c is read from buffer c % 2 while chunk c + 1 is written to the
    // other one; one barrier per chunk orders both
    auto stage = [&](int buf) {
#pragma unroll
        for (int e = 0; e < XPT; ++e) xs[buf][xk + e][xr] = xv[e];
#pragma unroll
        for (int e = 0; e < WPT; ++e) ws[buf][wk][wcol + e] = wv[e];
    };
    fetch(0);
    stage(0);
    __syncthreads();
    int buf = 0;
    for (int64_t k0 = 0; k0 < S; k0 += BK) {
        const bool more = k0 + BK < S;
        if (more) fetch(k0 + BK);
        const int ar = lane & 15, ak = lane >> 4;
#pragma unroll
        for (int kk = 0; kk < BK; kk += 4) {
            double a[TI], b[TJ];
#pragma unroll
            for (int i = 0; i < TI; ++i) a[i] = xs[buf][kk + ak][wr + i * 16 + ar];
#pragma unroll
            for (int j = 0; j < TJ; ++j) b[j] = ws[buf][kk + ak][wc + j * 16 + ar];
#pragma unroll
            for (int i = 0; i < TI; ++i)
#pragma unroll
                for (int j = 0; j < TJ; ++j)
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
        }
        if (more) stage(buf ^ 1);
        __syncthreads();
        buf ^= 1;
    }
    // epilogue: element r of a lane is row lane / 16 + 4 r of column lane % 16
    const int oc = lane & 15, orow = lane >> 4;
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) {
            const int64_t c = col0 + wc + j * 16 + oc;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t n = row0 + wr + i * 16 + orow + 4 * r;
                if (!full && (c >= K || n >= N)) continue;
                double* y = Y + n * ldy + c;
                if constexpr (ACC) *y += acc[i][j][r];
                else __builtin_nontemporal_store(acc[i][j][r], y);  // written once, not re-read here
            }
        }
}

}  // namespace
}  // namespace cut

using namespace cut;

extern "C" cut_status cut_assemble(const double* X, int64_t ldx, int64_t N, int64_t S, const double* W,
                                   int64_t ldw, int64_t K, double* Y, int64_t ldy, uint32_t flags,
                                   void* stream) {
    ABI_BEGIN
    if (N < 0 || S < 1 || K < 1) CUT_FAIL(CUT_E_INVAL, "cut_assemble: bad sizes");
    if (!X || !W || !Y) CUT_FAIL(CUT_E_INVAL, "cut_assemble: null operand");
    if (ldx < S || ldw < K || ldy < K) CUT_FAIL(CUT_E_INVAL, "cut_assemble: leading dimension too small");
    if ((flags & ~CUT_ACCUMULATE) != 0) CUT_FAIL(CUT_E_INVAL, "cut_assemble: unknown flags");
    if (N == 0) return CUT_OK;
    // 128 x 128 blocks (64 x 64 per wavefront), chunks of 8 sources: measured
    // at N = 92,170, S = 120, K = 1,024 against 64 x 64 and 128 x 64 blocks
    // and chunks of 4 and 16; row blocks along x (up to 2^31 - 1), column
    // blocks along y (up to 65535)
    constexpr int BM = 128, BN = 128, BK = 8;
    const int64_t gx = (N + BM - 1) / BM, gy = (K + BN - 1) / BN;
    if (gx > 0x7fffffff || gy > 65535) CUT_FAIL(CUT_E_INVAL, "cut_assemble: too large");
    const dim3 grid((unsigned)gx, (unsigned)gy);
    if (flags & CUT_ACCUMULATE)
        hipLaunchKernelGGL((k_assemble<BM, BN, BK, true>), grid, dim3(256), 0, (hipStream_t)stream, X, ldx, N, S, W,
                           ldw, K, Y, ldy);
    else
        hipLaunchKernelGGL((k_assemble<BM, BN, BK, false>), grid, dim3(256), 0, (hipStream_t)stream, X, ldx, N, S, W,
                           ldw, K, Y, ldy);
    HIP_CHECK(hipGetLastError());
    ABI_END
}
