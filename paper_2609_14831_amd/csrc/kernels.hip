// gfx950 kernels of the compiled-CUT-graph path.
//
// k_pass: segmented gather-multiply-reduce over one target-grouped record
// stream (Sec. 2.2: records that contribute to the same output are stored
// together and reduced directly into it).  One wavefront owns one output
// segment (or a quarter of a long one); its 64 lanes are split into R = 64/G
// record slots x G coefficient sets, so every gather is a contiguous run of G
// sets of one operand row.  Reductions are fixed-order (butterfly shuffles,
// then an ordered LDS combine for split segments): results are bitwise
// reproducible run to run.
//
//   MODE_BCAST : out[seg][op][s] = sum_e c_e * A[a_e][s] * B[b_e][op][s]
//                (forward action with a=i, b=j; adjoint-x with a=i, b=k)
//   MODE_REDOPS: out[seg][s]     = sum_e c_e * sum_op A[a_e][op][s] * B[b_e][op][s]
//                (adjoint-eta with a=k, b=j)
//
// Epilogues: EPI_Y (store / accumulate a double result, scaled), EPI_ETA
// (generator graph pass: store eta in the stage precision), EPI_RK (classic RK4
// stage combination fused into the flow pass, Eq. coflow integrated at fixed ds).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>

#include "internal.h"

namespace cut {

struct KArgs {
    const Task* tasks;
    int64_t ntasks;
    int64_t per_xcd;  // >0: task = (bid % 8) * per_xcd + bid / 8
    const int64_t* off;
    const uint2* rec;
    const void* A;
    int64_t lda;
    const void* B;
    int64_t ldb;
    int32_t nsets, nops;
    int32_t s0, s1;   // the sets [s0, s1) this launch covers (columns keep the nsets stride)
    const int32_t* nsteps;
    const int32_t* step;
    void* y;
    int64_t ldy;
    int32_t accumulate;
    int32_t out_f32;
    double scale;
    int32_t stage;
    double ds;
    double* z;
    double* acc;
    void* xout;
    double* hst;
    int64_t ldh;
    // chunk tasks (long segments): partial rows instead of the epilogue
    const ChunkTask* chunks;
    int64_t nchunks;
    int64_t nchunk_blocks;  // blocks [0, nchunk_blocks) take chunks, the rest `tasks`
    double* part;
    int64_t ldp;
    // both operand arrays span less than 2 GiB: gathers address rows by a
    // 32-bit scalar offset from one buffer resource per array
    int32_t buf32;
};

template <int PREC>
struct PrecT {
    using T = float;
};
template <>
struct PrecT<CUT_F64> {
    using T = double;
};

// Accumulator of one lane for one operand column.
template <int PREC>
struct Acc;

template <>
struct Acc<CUT_F64> {
    double v = 0.0;
    __device__ void add(double t, double b) { v = __builtin_fma(t, b, v); }
    __device__ double get() const { return v; }
};
template <>
struct Acc<CUT_F32X> {
    double v = 0.0;
    __device__ void add(double t, float b) { v = __builtin_fma(t, (double)b, v); }
    __device__ double get() const { return v; }
};
template <>
struct Acc<CUT_F32> {
    float v = 0.f;
    __device__ void add(float t, float b) { v = __builtin_fmaf(t, b, v); }
    __device__ double get() const { return (double)v; }
};
// Compensated: error-free product (FMA) and error-free sum (two-sum); the
// running error terms are summed in a second float.  add() treats one term;
// add_sum() folds the float partial of a group of terms (accumulated by FMAs,
// so its products and sums are rounded within the group only) into (hi, lo)
// with one two-sum: per term that costs one FMA plus 1/U of the two-sum.
template <>
struct Acc<CUT_F32C> {
    float hi = 0.f, lo = 0.f;
    __device__ void add(float t, float b) {
        // the error-free transformations need every operation rounded on its
        // own: no contraction of t*b into the following additions
#pragma clang fp contract(off)
        float p = t * b;
        float pe = __builtin_fmaf(t, b, -p);
        float s = hi + p;
        float bb = s - hi;
        float se = (hi - (s - bb)) + (p - bb);
        hi = s;
        lo += se + pe;
    }
    __device__ void add_sum(float p) {
#pragma clang fp contract(off)
        float s = hi + p;
        float bb = s - hi;
        float se = (hi - (s - bb)) + (p - bb);
        hi = s;
        lo += se;
    }
    __device__ double get() const { return (double)hi + (double)lo; }
};

// scaled left operand in the accumulation type
template <int PREC>
__device__ inline auto left_term(double cf, typename PrecT<PREC>::T av) {
    if constexpr (PREC == CUT_F64) return cf * av;
    else if constexpr (PREC == CUT_F32X) return cf * (double)av;
    else return (float)cf * av;
}

// acc[op] += sum_u t[u] * b[u][op]: in the compensated float mode the U terms
// of a column share one float partial and one two-sum; otherwise term by term
template <int PREC, int U, int NOPS, class TL, class TB>
__device__ inline void add_group(Acc<PREC> (&acc)[NOPS], const TL (&t)[U], const TB (&b)[U][NOPS]) {
    if constexpr (PREC == CUT_F32C) {
#pragma unroll
        for (int op = 0; op < NOPS; ++op) {
            float p = t[0] * b[0][op];
#pragma unroll
            for (int u = 1; u < U; ++u) p = __builtin_fmaf(t[u], b[u][op], p);
            acc[op].add_sum(p);
        }
    } else {
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int op = 0; op < NOPS; ++op) acc[op].add(t[u], b[u][op]);
    }
}

// FP32 bit pattern of the factor of a device record: its bf16 bit pattern is
// split over the top bytes of the two row indices (high byte with the left row).
__device__ __forceinline__ uint32_t record_factor_bits(uint32_t x, uint32_t y) {
    return (x & 0xFF000000u) | ((y >> 24) << 16);
}

__device__ __forceinline__ int64_t uniform64(int64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Gather of one element of a row through a buffer resource built (on the
// scalar unit) from the uniform row address: the lane's byte offset is the only
// per-lane operand, so a gather costs no vector address arithmetic.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t row_rsrc(const void* row, int64_t bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(row), (short)0, (int)bytes, 0x00020000);
}
template <class T>
__device__ __forceinline__ T buf_load(__amdgpu_buffer_rsrc_t r, uint32_t voff, int32_t soff) {
    if constexpr (sizeof(T) == 4) {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, soff, 0));
    } else {
        return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, soff, 0));
    }
}

__device__ inline bool set_active(const KArgs& a, int s) {
    if (s >= a.nsets) return false;
    if (a.nsteps == nullptr) return true;
    return a.nsteps[s] > *a.step;
}

// Classic RK4 stage combination for the NOPS operand values f of row `seg`,
// set s: stage 0 starts the accumulator, 1-2 add to it, 3 finishes the step;
// the next stage operand is written (float or double shadow) together with the
// FP64 Hamiltonian column.  z and the accumulator are touched once per stage:
// streamed with non-temporal hints so they do not displace gathered rows.
// One state element idx with right-hand side f at stage a.stage: updates the
// accumulator (and, at the last stage, z) and returns the next stage state.
__device__ inline double rk_combine(const KArgs& a, int64_t idx, double f) {
    const double ds = a.ds;
    const double zk = __builtin_nontemporal_load(a.z + idx);
    double nxt;
    if (a.stage == 0) {
        __builtin_nontemporal_store(zk + (ds / 6.0) * f, a.acc + idx);
        nxt = zk + 0.5 * ds * f;
    } else if (a.stage == 1) {
        __builtin_nontemporal_store(__builtin_nontemporal_load(a.acc + idx) + (ds / 3.0) * f, a.acc + idx);
        nxt = zk + 0.5 * ds * f;
    } else if (a.stage == 2) {
        __builtin_nontemporal_store(__builtin_nontemporal_load(a.acc + idx) + (ds / 3.0) * f, a.acc + idx);
        nxt = zk + ds * f;
    } else {
        nxt = __builtin_nontemporal_load(a.acc + idx) + (ds / 6.0) * f;
        __builtin_nontemporal_store(nxt, a.z + idx);
    }
    return nxt;
}

template <int NOPS, class T>
__device__ inline void rk_epilogue(const KArgs& a, int64_t seg, int s, const double* v) {
    T* xo = (T*)a.xout;
#pragma unroll
    for (int op = 0; op < NOPS; ++op) {
        const int64_t idx = seg * a.ldb + (int64_t)op * a.nsets + s;
        const double nxt = rk_combine(a, idx, v[op]);
        xo[idx] = (T)nxt;
        if (op == 0) a.hst[seg * a.ldh + s] = nxt;
    }
}

template <int G, int NOPS, int PREC, int MODE, int EPI>
__global__ __launch_bounds__(256) void k_pass(KArgs a) {
    using T = typename PrecT<PREC>::T;
    constexpr int R = 64 / G;
    constexpr int NACC = (MODE == MODE_REDOPS) ? 1 : NOPS;
    __shared__ double red[4][NACC][G];

    // wave index through an SGPR so segment bounds and loop control stay scalar
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int sg = lane % G;
    const int sub = lane / G;
    const int s = a.s0 + blockIdx.y * G + sg;
    const bool act = s < a.s1 && set_active(a, s);
    const bool chunked = a.chunks != nullptr && (int64_t)blockIdx.x < a.nchunk_blocks;
    Task task{0, 0};
    int32_t slot = 0;
    int64_t seg, e0, e1;
    if (chunked) {  // one chunk of a long segment per wavefront
        const int64_t ci = (int64_t)blockIdx.x * 4 + wave;
        if (ci >= a.nchunks) return;
        const ChunkTask ct = a.chunks[ci];
        if (ct.seg < 0) return;  // padding of the XCD split
        seg = ct.seg;
        slot = ct.slot;
        e0 = ct.e0;
        e1 = ct.e1;
    } else {
        // nchunk_blocks is a multiple of 8, so b keeps the XCD of the block
        const int64_t b = (int64_t)blockIdx.x - (a.chunks ? a.nchunk_blocks : 0);
        int64_t t = b;
        if (a.per_xcd > 0) {
            t = (b & 7) * a.per_xcd + (b >> 3);
            if ((b >> 3) >= a.per_xcd) return;
        }
        if (t >= a.ntasks) return;
        task = a.tasks[t];
    }
    const bool split = !chunked && task.nseg < 0;

    if (chunked) {
    } else if (split) {
        seg = task.seg;
        const int64_t b = a.off[seg], n = a.off[seg + 1] - b;
        e0 = b + (n * wave) / 4;
        e1 = b + (n * (wave + 1)) / 4;
    } else {
        if (wave >= task.nseg) return;  // block-uniform task kind: no barrier below
        seg = task.seg + wave;
        e0 = a.off[seg];
        e1 = a.off[seg + 1];
    }

    // segment bounds are wavefront-uniform: keep them (and the loop control
    // derived from them) on the scalar unit
    e0 = uniform64(e0);
    e1 = uniform64(e1);
    Acc<PREC> acc[NACC];
    const T* __restrict__ A = (const T*)a.A;
    const T* __restrict__ B = (const T*)a.B;
    const int nsets = a.nsets;
    // lanes of inactive sets compute on an in-range column and are discarded
    // at the epilogue; no load is ever predicated
    const int sl = s < a.s1 ? s : a.s1 - 1;
    // lane byte offsets of the gathered columns within a row: 32-bit and
    // unsigned, so each gather takes the (uniform) row address as its scalar
    // base and needs no per-lane address arithmetic
    uint32_t boff[NOPS];
#pragma unroll
    for (int op = 0; op < NOPS; ++op) boff[op] = (uint32_t)(sl + op * nsets) * (uint32_t)sizeof(T);
    constexpr int NA = (MODE == MODE_REDOPS) ? NOPS : 1;
#ifndef CUT_PASS_UNROLL
#define CUT_PASS_UNROLL 4
#endif
    constexpr int U = (PREC == CUT_F32C && G == 32) ? 16 : (NOPS <= 2 || PREC == CUT_F32C) ? 8 : CUT_PASS_UNROLL;
    // The gathers of U records are all issued before any arithmetic, so U
    // dependent load chains are in flight per lane group; then accum() adds the
    // U terms.  A record slot past the segment end holds a valid clamped record
    // and gets factor zero.  Compensated-float passes with 32-lane groups take
    // U = 16 (measured 3 % faster than 8; the float partial of a group then
    // carries at most gamma_16 of its terms).
    auto accum = [&](const T (&av)[U][NA], const T (&bv)[U][NOPS], const float (&fc)[U]) {
        if constexpr (PREC == CUT_F32C) {
            // the U terms of each column in one float partial (FMA chain),
            // then one two-sum into the compensated accumulator
            if constexpr (MODE == MODE_BCAST) {
                float tl[U];
#pragma unroll
                for (int u = 0; u < U; ++u) tl[u] = fc[u] * av[u][0];
#pragma unroll
                for (int op = 0; op < NOPS; ++op) {
                    float p = tl[0] * bv[0][op];
#pragma unroll
                    for (int u = 1; u < U; ++u) p = __builtin_fmaf(tl[u], bv[u][op], p);
                    acc[op].add_sum(p);
                }
            } else {
                float p = 0.f;
#pragma unroll
                for (int u = 0; u < U; ++u)
#pragma unroll
                    for (int op = 0; op < NOPS; ++op) p = __builtin_fmaf(fc[u] * av[u][op], bv[u][op], p);
                acc[0].add_sum(p);
            }
            return;
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double cf = (double)fc[u];
            if constexpr (MODE == MODE_BCAST && PREC == CUT_F32) {
                const float tl = fc[u] * av[u][0];
#pragma unroll
                for (int op = 0; op < NOPS; ++op) acc[op].add(tl, bv[u][op]);
            } else if constexpr (MODE == MODE_BCAST) {
                const auto tl = left_term<PREC>(cf, av[u][0]);
#pragma unroll
                for (int op = 0; op < NOPS; ++op) acc[op].add(tl, bv[u][op]);
            } else if constexpr (PREC == CUT_F64 || PREC == CUT_F32X) {
                // sum over operand columns first, then one scaled accumulation
                double d = 0.0;
#pragma unroll
                for (int op = 0; op < NOPS; ++op) d = __builtin_fma((double)av[u][op], (double)bv[u][op], d);
                acc[0].v = __builtin_fma(cf, d, acc[0].v);
            } else {
#pragma unroll
                for (int op = 0; op < NOPS; ++op) acc[0].add(fc[u] * av[u][op], bv[u][op]);
            }
        }
    };
    // records given as (x, y) words; okm[u] all ones for a live slot, else zero
    auto consume = [&](const uint32_t (&rx)[U], const uint32_t (&ry)[U], const uint32_t (&okm)[U]) {
        T av[U][NA];
        T bv[U][NOPS];
        float fc[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            // 24-bit row index times a 32-bit stride (checked on the host):
            // one 32 x 32 -> 64-bit multiply-add per row
            const T* arow = A + (uint64_t)(rx[u] & 0xFFFFFFu) * (uint32_t)a.lda;
            const T* brow = B + (uint64_t)(ry[u] & 0xFFFFFFu) * (uint32_t)a.ldb;
            fc[u] = __builtin_bit_cast(float, record_factor_bits(rx[u], ry[u]) & okm[u]);
            if constexpr (G == 64) {  // one record per wavefront: uniform rows
                const auto ra = row_rsrc(arow, a.lda * (int64_t)sizeof(T));
                const auto rb = row_rsrc(brow, a.ldb * (int64_t)sizeof(T));
#pragma unroll
                for (int q = 0; q < NA; ++q) av[u][q] = buf_load<T>(ra, boff[q], 0);
#pragma unroll
                for (int op = 0; op < NOPS; ++op) bv[u][op] = buf_load<T>(rb, boff[op], 0);
            } else if constexpr (G == 1) {
                if (nsets == 1) {
                    // one set: a row's columns are contiguous at offsets known
                    // at compile time, so the compiler fuses them into 16-byte
                    // loads (half the per-lane gather instructions)
#pragma unroll
                    for (int q = 0; q < NA; ++q) av[u][q] = arow[q];
#pragma unroll
                    for (int op = 0; op < NOPS; ++op) bv[u][op] = brow[op];
                } else {
                    // one set of several (a one-set piece of a set range)
                    const char* ac = reinterpret_cast<const char*>(arow);
                    const char* bc = reinterpret_cast<const char*>(brow);
#pragma unroll
                    for (int q = 0; q < NA; ++q) av[u][q] = *reinterpret_cast<const T*>(ac + boff[q]);
#pragma unroll
                    for (int op = 0; op < NOPS; ++op) bv[u][op] = *reinterpret_cast<const T*>(bc + boff[op]);
                }
            } else {
                const char* ac = reinterpret_cast<const char*>(arow);
                const char* bc = reinterpret_cast<const char*>(brow);
#pragma unroll
                for (int q = 0; q < NA; ++q) av[u][q] = *reinterpret_cast<const T*>(ac + boff[q]);
#pragma unroll
                for (int op = 0; op < NOPS; ++op) bv[u][op] = *reinterpret_cast<const T*>(bc + boff[op]);
            }
        }
        accum(av, bv, fc);
    };
    if constexpr (G == 64) {
        // One record per wavefront step: records come through scalar loads
        // (uniform index, read-only stream).  32-bit positions within the
        // segment keep the compares scalar (no scalar 64-bit signed compare).
        typedef const __attribute__((address_space(4))) unsigned long long ConstRec;
        const ConstRec* rp = (const ConstRec*)a.rec + e0;
        const int32_t n = (int32_t)(e1 - e0);
        // records q0 .. q0+U-1 (clamped to the last one past the end; no branch,
        // so the loads stay in flight across the code that follows)
        auto fetch = [&](int32_t q0, uint32_t (&x)[U], uint32_t (&y)[U]) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t q = q0 + u < n ? q0 + u : n - 1;
                const unsigned long long r = rp[q];
                x[u] = (uint32_t)r;
                y[u] = (uint32_t)(r >> 32);
            }
        };
        auto live = [&](int32_t b, uint32_t (&okm)[U]) {
#pragma unroll
            for (int u = 0; u < U; ++u) okm[u] = ~(uint32_t)((n - 1 - (b + u)) >> 31);  // integer ops: scalar
        };
        if (a.buf32) {
            // Both operand arrays below 2 GiB: one buffer resource per array,
            // rows addressed by 32-bit scalar offsets.  Scalar loads complete
            // out of order, so any use of one group's records waits for every
            // scalar load in flight: each group's offsets and factors are
            // derived first, and only then (past a scheduling barrier) are the
            // records of the group after next fetched into the same registers.
            const auto rsA = row_rsrc(A, 0x7FFFFFFF);
            const auto rsB = row_rsrc(B, 0x7FFFFFFF);
            const int32_t lda_b = (int32_t)(a.lda * (int64_t)sizeof(T));
            const int32_t ldb_b = (int32_t)(a.ldb * (int64_t)sizeof(T));
            auto group = [&](int32_t b, uint32_t (&x)[U], uint32_t (&y)[U]) {
                uint32_t okm[U];
                live(b, okm);
                int32_t sa[U], sb[U];
                float fc[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    sa[u] = (int32_t)(x[u] & 0xFFFFFFu) * lda_b;
                    sb[u] = (int32_t)(y[u] & 0xFFFFFFu) * ldb_b;
                    fc[u] = __builtin_bit_cast(float, record_factor_bits(x[u], y[u]) & okm[u]);
                }
                __builtin_amdgcn_sched_barrier(0);
                fetch(b + 2 * U, x, y);
                T av[U][NA];
                T bv[U][NOPS];
#pragma unroll
                for (int u = 0; u < U; ++u) {
#pragma unroll
                    for (int q = 0; q < NA; ++q) av[u][q] = buf_load<T>(rsA, boff[q], sa[u]);
#pragma unroll
                    for (int op = 0; op < NOPS; ++op) bv[u][op] = buf_load<T>(rsB, boff[op], sb[u]);
                }
                accum(av, bv, fc);
            };
            uint32_t xa[U], ya[U], xb[U], yb[U];
            if (n > 0) fetch(0, xa, ya);
            if (n > U) fetch(U, xb, yb);
            for (int32_t b = 0; b < n; b += 2 * U) {
                group(b, xa, ya);
                if (b + U >= n) break;
                group(b + U, xb, yb);
            }
        } else {
            uint32_t rx[U], ry[U];
            for (int32_t b = 0; b < n; b += U) {
                fetch(b, rx, ry);
                uint32_t okm[U];
                live(b, okm);
                consume(rx, ry, okm);
            }
        }
    } else {
        // Records are fetched cooperatively, 64 per wavefront load (one per
        // lane), then handed to the lane groups by cross-lane moves.
        constexpr int CH = (G >= U) ? 2 : U / G;  // 64-record chunks per outer iteration
        constexpr int SLOTS = CH * G;             // record slots of one lane group per iteration
        __shared__ uint2 recs[4][G > 1 ? 64 * CH : 1];
        for (int64_t base = e0; base < e1; base += 64 * CH) {
            uint2 mine[CH];
#pragma unroll
            for (int c = 0; c < CH; ++c) {
                // clamped (always valid) address; slots past e1 are masked by cnt
                const int64_t idx = base + c * 64 + lane;
                // records are read once per pass: non-temporal
                const unsigned long long rv = __builtin_nontemporal_load(
                    (const unsigned long long*)a.rec + (idx < e1 ? idx : e1 - 1));
                mine[c] = make_uint2((uint32_t)rv, (uint32_t)(rv >> 32));
            }
            const int cnt = (int)((e1 - base) < 64 * CH ? (e1 - base) : 64 * CH);
            if constexpr (G > 1) {
                // the wavefront's records go through its own LDS slice: slot t
                // of lane group `sub` is record t R + sub, one broadcast read
                // per slot (LDS operations of one wavefront complete in order;
                // the fences keep the compiler from moving reads above writes
                // or the next writes above reads)
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
#pragma unroll
                for (int c = 0; c < CH; ++c) recs[wave][c * 64 + lane] = mine[c];
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            }
#pragma unroll
            for (int t0 = 0; t0 < SLOTS; t0 += U) {
                if (t0 * R >= cnt) break;
                uint32_t rx[U], ry[U], okm[U];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const int t = t0 + u;
                    const int c = t / G;
                    if constexpr (G == 1) {  // every lane takes its own record
                        rx[u] = mine[c].x;
                        ry[u] = mine[c].y;
                    } else {
                        const uint2 r = recs[wave][t * R + sub];
                        rx[u] = r.x;
                        ry[u] = r.y;
                    }
                    okm[u] = t * R + sub < cnt ? 0xFFFFFFFFu : 0u;
                }
                consume(rx, ry, okm);
            }
        }
    }

    double v[NACC];
#pragma unroll
    for (int q = 0; q < NACC; ++q) {
        v[q] = acc[q].get();
#pragma unroll
        for (int o = G; o < 64; o <<= 1) v[q] += __shfl_xor(v[q], o);
    }
    if (chunked) {
        if (sub == 0 && act) {
            double* p = a.part + (int64_t)slot * a.ldp + s;
#pragma unroll
            for (int q = 0; q < NACC; ++q) p[(int64_t)q * nsets] = v[q];
        }
        return;
    }
    if (split) {
        if (sub == 0) {
#pragma unroll
            for (int q = 0; q < NACC; ++q) red[wave][q][sg] = v[q];
        }
        __syncthreads();
        if (wave != 0) return;
#pragma unroll
        for (int q = 0; q < NACC; ++q) {
            if (sub == 0) v[q] = ((red[0][q][sg] + red[1][q][sg]) + red[2][q][sg]) + red[3][q][sg];
        }
    }
    if (sub != 0 || !act) return;

    if constexpr (EPI == EPI_Y) {
        double* y = (double*)a.y + seg * a.ldy + s;
        if constexpr (MODE == MODE_REDOPS) {
            y[0] = a.accumulate ? y[0] + a.scale * v[0] : a.scale * v[0];
        } else {
#pragma unroll
            for (int op = 0; op < NOPS; ++op) {
                double& o = y[(int64_t)op * nsets];
                o = a.accumulate ? o + a.scale * v[op] : a.scale * v[op];
            }
        }
    } else if constexpr (EPI == EPI_ETA) {
        if (a.out_f32) ((float*)a.y)[seg * a.ldy + s] = (float)(a.scale * v[0]);
        else ((double*)a.y)[seg * a.ldy + s] = a.scale * v[0];
    } else {  // EPI_RK: stage combination of classic RK4
        rk_epilogue<NOPS, T>(a, seg, s, v);
    }
}

// ------------------------------------------------ complex-record pass ----
// Pauli-boson graphs, FP64 forward passes straight over the complex records
// (Sec. 2.2, Eq. graph-actions, with Gaussian-integer factors that are purely
// real or purely imaginary).  Record: x = (f_hi << 24) | (imag << 23) | a,
// y = (f_lo << 24) | j, (f_hi, f_lo) the bf16 pattern of the nonzero part of
// the factor; a is a complex generator row (real-split rows 2a, 2a + 1 of A),
// j a complex operand row (rows 2j, 2j + 1 of B).  One record occupies NCP
// lanes, lane = (slot q, column c), NCP the column count nops * nsets rounded
// up to a power of two; each lane gathers the generator entry (both parts) and
// both rows of its column of x_j and sums the real and the imaginary part of
// the target:  g x = (g_r x_r - g_i x_i) + i (g_r x_i + g_i x_r), times f for
// a real factor, times i f for an imaginary one.  One complex record is read
// once for its four real products, from a record stream a quarter the size of
// the real-split one.  Targets are the segments of the complex CSR; tasks are
// planned like the real-split ones (short targets one per wavefront, long ones
// split over the 4 wavefronts of a workgroup and combined in LDS in fixed
// order).
// GPAIR: the generator has one column at unit stride, so both parts of an
// entry are one 16-byte load.  Operand offsets are 32-bit byte offsets from
// the array base (the host checks that both arrays span less than 4 GiB).
template <int NCP, int EPI, bool GPAIR>
__global__ __launch_bounds__(256) void k_cpass(KArgs a) {
    constexpr int RS = 64 / NCP, U = 4;
    __shared__ double red[4][2][64];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int q = lane / NCP, c = lane % NCP;
    const int nsets = a.nsets, ncol = a.nops * nsets;
    const int cc = c < ncol ? c : ncol - 1;  // lanes past the last column compute on a valid one
    const int s = nsets == 1 ? 0 : cc % nsets;
    const int64_t b = blockIdx.x;
    int64_t t = b;
    if (a.per_xcd > 0) {
        t = (b & 7) * a.per_xcd + (b >> 3);
        if ((b >> 3) >= a.per_xcd) return;
    }
    if (t >= a.ntasks) return;
    const Task task = a.tasks[t];
    const bool split = task.nseg < 0;
    int64_t seg, e0, e1;
    if (split) {
        seg = task.seg;
        const int64_t b0 = a.off[seg], n = a.off[seg + 1] - b0;
        e0 = b0 + (n * wave) / 4;
        e1 = b0 + (n * (wave + 1)) / 4;
    } else {
        if (wave >= task.nseg) return;  // block-uniform task kind: no barrier below
        seg = task.seg + wave;
        e0 = a.off[seg];
        e1 = a.off[seg + 1];
    }
    e0 = uniform64(e0);
    e1 = uniform64(e1);
    const char* __restrict__ A = (const char*)a.A;
    const char* __restrict__ B = (const char*)a.B;
    const uint32_t lda8 = (uint32_t)a.lda * 8u, ldb8 = (uint32_t)a.ldb * 8u;
    const uint32_t aoff = (uint32_t)s * 8u, boff = (uint32_t)cc * 8u;
    const uint2* __restrict__ rec = a.rec;
    auto fetch = [&](int64_t base, uint2 (&r)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = base + u * RS + q;
            r[u] = rec[e < e1 ? e : e1 - 1];  // clamped: always a valid record
        }
    };
    double are = 0.0, aim = 0.0;
    uint2 r[U];
    if (e0 < e1) fetch(e0, r);
    for (int64_t base = e0; base < e1; base += RS * U) {
        double gr[U], gi[U], xr[U], xi[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const uint32_t ga = 2u * (r[u].x & 0x7FFFFFu) * lda8 + aoff;
            if constexpr (GPAIR) {
                const double2 gv = *reinterpret_cast<const double2*>(A + ga);
                gr[u] = gv.x;
                gi[u] = gv.y;
            } else {
                gr[u] = *reinterpret_cast<const double*>(A + ga);
                gi[u] = *reinterpret_cast<const double*>(A + (ga + lda8));
            }
            const uint32_t xb = 2u * (r[u].y & 0xFFFFFFu) * ldb8 + boff;
            xr[u] = *reinterpret_cast<const double*>(B + xb);
            xi[u] = *reinterpret_cast<const double*>(B + (xb + ldb8));
        }
        uint32_t fb[U], im[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            im[u] = (r[u].x >> 23) & 1u;
            fb[u] = base + u * RS + q < e1 ? record_factor_bits(r[u].x, r[u].y) : 0u;
        }
        if (base + RS * U < e1) fetch(base + RS * U, r);  // next group's records in flight
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double f = (double)__builtin_bit_cast(float, fb[u]);
            const double pr = __builtin_fma(-gi[u], xi[u], gr[u] * xr[u]);
            const double pi = __builtin_fma(gi[u], xr[u], gr[u] * xi[u]);
            are = __builtin_fma(f, im[u] ? -pi : pr, are);
            aim = __builtin_fma(f, im[u] ? pr : pi, aim);
        }
    }
#pragma unroll
    for (int o = NCP; o < 64; o <<= 1) {
        are += __shfl_xor(are, o);
        aim += __shfl_xor(aim, o);
    }
    if (split) {
        if (q == 0) {
            red[wave][0][lane] = are;
            red[wave][1][lane] = aim;
        }
        __syncthreads();
        if (wave != 0) return;
        if (q == 0) {
            are = ((red[0][0][lane] + red[1][0][lane]) + red[2][0][lane]) + red[3][0][lane];
            aim = ((red[0][1][lane] + red[1][1][lane]) + red[2][1][lane]) + red[3][1][lane];
        }
    }
    if (q != 0 || c >= ncol || !set_active(a, s)) return;
    const int64_t ldb = a.ldb;
#pragma unroll
    for (int part = 0; part < 2; ++part) {
        const int64_t row = 2 * seg + part;
        const double v = part ? aim : are;
        if constexpr (EPI == EPI_Y) {
            double* y = (double*)a.y + row * a.ldy + c;
            *y = a.accumulate ? *y + a.scale * v : a.scale * v;
        } else {
            const double nxt = rk_combine(a, row * ldb + c, v);
            ((double*)a.xout)[row * ldb + c] = nxt;
            if (c < nsets) a.hst[row * a.ldh + s] = nxt;  // operand 0 = the Hamiltonian
        }
    }
}

// k_cpass for one coefficient set, a column count divisible by CPL (2 or 4), a
// one-column generator at unit stride and 16-byte aligned operand rows: every
// lane takes CPL adjacent columns (16-byte loads of both rows of x_j), so a
// record occupies NCP / CPL lanes and a wavefront step holds CPL times as many
// records as in k_cpass (fewer load instructions per record).
template <int NCP, int EPI, int CPL>
__global__ __launch_bounds__(256) void k_cpassw(KArgs a) {
    constexpr int LPR = NCP / CPL, RS = 64 / LPR, U = CPL == 2 ? 4 : 2;
    static_assert(CPL == 2 || CPL == 4, "columns per lane");
    __shared__ double red[4][2 * CPL][64];
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int q = lane / LPR, cl = lane % LPR;
    const int ncol = a.nops;                                   // one set: columns = operands
    const int c0 = CPL * cl < ncol ? CPL * cl : ncol - CPL;    // lanes past the last group compute on a valid one
    const int64_t b = blockIdx.x;
    int64_t t = b;
    if (a.per_xcd > 0) {
        t = (b & 7) * a.per_xcd + (b >> 3);
        if ((b >> 3) >= a.per_xcd) return;
    }
    if (t >= a.ntasks) return;
    const Task task = a.tasks[t];
    const bool split = task.nseg < 0;
    int64_t seg, e0, e1;
    if (split) {
        seg = task.seg;
        const int64_t b0 = a.off[seg], n = a.off[seg + 1] - b0;
        e0 = b0 + (n * wave) / 4;
        e1 = b0 + (n * (wave + 1)) / 4;
    } else {
        if (wave >= task.nseg) return;  // block-uniform task kind: no barrier below
        seg = task.seg + wave;
        e0 = a.off[seg];
        e1 = a.off[seg + 1];
    }
    e0 = uniform64(e0);
    e1 = uniform64(e1);
    const char* __restrict__ A = (const char*)a.A;
    const char* __restrict__ B = (const char*)a.B;
    const uint32_t ldb8 = (uint32_t)a.ldb * 8u, boff = (uint32_t)c0 * 8u;
    const uint2* __restrict__ rec = a.rec;
    auto fetch = [&](int64_t base, uint2 (&r)[U]) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t e = base + u * RS + q;
            r[u] = rec[e < e1 ? e : e1 - 1];  // clamped: always a valid record
        }
    };
    double are[CPL], aim[CPL];
#pragma unroll
    for (int h = 0; h < CPL; ++h) are[h] = aim[h] = 0.0;
    uint2 r[U];
    if (e0 < e1) fetch(e0, r);
    for (int64_t base = e0; base < e1; base += RS * U) {
        double2 gv[U], xr[U][CPL / 2], xi[U][CPL / 2];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            gv[u] = *reinterpret_cast<const double2*>(A + 16u * (r[u].x & 0x7FFFFFu));
            const uint32_t xb = 2u * (r[u].y & 0xFFFFFFu) * ldb8 + boff;
#pragma unroll
            for (int h = 0; h < CPL / 2; ++h) {
                xr[u][h] = *reinterpret_cast<const double2*>(B + (xb + 16u * h));
                xi[u][h] = *reinterpret_cast<const double2*>(B + (xb + ldb8 + 16u * h));
            }
        }
        uint32_t fb[U], im[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            im[u] = (r[u].x >> 23) & 1u;
            fb[u] = base + u * RS + q < e1 ? record_factor_bits(r[u].x, r[u].y) : 0u;
        }
        if (base + RS * U < e1) fetch(base + RS * U, r);  // next group's records in flight
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double f = (double)__builtin_bit_cast(float, fb[u]);
            const double gr = gv[u].x, gi = gv[u].y;
#pragma unroll
            for (int h = 0; h < CPL; ++h) {
                const double vr = (h & 1) ? xr[u][h / 2].y : xr[u][h / 2].x;
                const double vi = (h & 1) ? xi[u][h / 2].y : xi[u][h / 2].x;
                const double pr = __builtin_fma(-gi, vi, gr * vr);
                const double pi = __builtin_fma(gi, vr, gr * vi);
                are[h] = __builtin_fma(f, im[u] ? -pi : pr, are[h]);
                aim[h] = __builtin_fma(f, im[u] ? pr : pi, aim[h]);
            }
        }
    }
#pragma unroll
    for (int o = LPR; o < 64; o <<= 1)
#pragma unroll
        for (int h = 0; h < CPL; ++h) {
            are[h] += __shfl_xor(are[h], o);
            aim[h] += __shfl_xor(aim[h], o);
        }
    if (split) {
        if (q == 0)
#pragma unroll
            for (int h = 0; h < CPL; ++h) {
                red[wave][2 * h][lane] = are[h];
                red[wave][2 * h + 1][lane] = aim[h];
            }
        __syncthreads();
        if (wave != 0) return;
        if (q == 0)
#pragma unroll
            for (int h = 0; h < CPL; ++h) {
                are[h] = ((red[0][2 * h][lane] + red[1][2 * h][lane]) + red[2][2 * h][lane]) + red[3][2 * h][lane];
                aim[h] = ((red[0][2 * h + 1][lane] + red[1][2 * h + 1][lane]) + red[2][2 * h + 1][lane]) +
                         red[3][2 * h + 1][lane];
            }
    }
    if (q != 0 || CPL * cl >= ncol || !set_active(a, 0)) return;
    const int64_t ldb = a.ldb;
#pragma unroll
    for (int part = 0; part < 2; ++part) {
        const int64_t row = 2 * seg + part;
#pragma unroll
        for (int h = 0; h < CPL; ++h) {
            const int c = c0 + h;
            const double v = part ? aim[h] : are[h];
            if constexpr (EPI == EPI_Y) {
                double* y = (double*)a.y + row * a.ldy + c;
                *y = a.accumulate ? *y + a.scale * v : a.scale * v;
            } else {
                const double nxt = rk_combine(a, row * ldb + c, v);
                ((double*)a.xout)[row * ldb + c] = nxt;
                if (c == 0) a.hst[row * a.ldh] = nxt;  // operand 0 = the Hamiltonian
            }
        }
    }
}

// Short complex targets (at most kShortMax records each, the generator set
// E_eta of a Pauli-boson graph: about 4 per target), several per wavefront:
// lane = (target slot, record slot q of 8, column c of NCP), so a wavefront
// takes 8 / NCP consecutive targets and a workgroup 4 times as many; no task
// list.  The arithmetic is that of k_cpass; the loop runs to the longest
// target of the wavefront, shorter ones with factor zero on a valid record.
constexpr int64_t kShortMax = 64;

template <int NCP, int EPI, bool GPAIR>
__global__ __launch_bounds__(256) void k_cshort(KArgs a, int64_t ntargets) {
    constexpr int RS = 8, LT = RS * NCP, TPW = 64 / LT;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int slot = lane / LT, q = (lane % LT) / NCP, c = lane % NCP;
    const int64_t k = ((int64_t)blockIdx.x * 4 + wave) * TPW + slot;
    const bool live = k < ntargets;
    const int64_t kk = live ? k : ntargets - 1;
    const int nsets = a.nsets, ncol = a.nops * nsets;
    const int cc = c < ncol ? c : ncol - 1;
    const int s = nsets == 1 ? 0 : cc % nsets;
    const int64_t e0 = a.off[kk], e1 = a.off[kk + 1];
    int n = (int)(e1 - e0);
#pragma unroll
    for (int o = LT; o < 64; o <<= 1) n = max(n, __shfl_xor(n, o));
    const char* __restrict__ A = (const char*)a.A;
    const char* __restrict__ B = (const char*)a.B;
    const uint32_t lda8 = (uint32_t)a.lda * 8u, ldb8 = (uint32_t)a.ldb * 8u;
    const uint32_t aoff = (uint32_t)s * 8u, boff = (uint32_t)cc * 8u;
    double are = 0.0, aim = 0.0;
    for (int base = 0; base < n; base += RS) {
        const int64_t e = e0 + base + q;
        const bool ok = e < e1;
        const uint2 r = a.rec[ok ? e : (e1 > e0 ? e1 - 1 : 0)];  // the host launches only when E > 0
        const uint32_t ga = 2u * (r.x & 0x7FFFFFu) * lda8 + aoff;
        double gr, gi;
        if constexpr (GPAIR) {
            const double2 gv = *reinterpret_cast<const double2*>(A + ga);
            gr = gv.x;
            gi = gv.y;
        } else {
            gr = *reinterpret_cast<const double*>(A + ga);
            gi = *reinterpret_cast<const double*>(A + (ga + lda8));
        }
        const uint32_t xb = 2u * (r.y & 0xFFFFFFu) * ldb8 + boff;
        const double xr = *reinterpret_cast<const double*>(B + xb);
        const double xi = *reinterpret_cast<const double*>(B + (xb + ldb8));
        const uint32_t im = (r.x >> 23) & 1u;
        const double f = ok ? (double)__builtin_bit_cast(float, record_factor_bits(r.x, r.y)) : 0.0;
        const double pr = __builtin_fma(-gi, xi, gr * xr);
        const double pi = __builtin_fma(gi, xr, gr * xi);
        are = __builtin_fma(f, im ? -pi : pr, are);
        aim = __builtin_fma(f, im ? pr : pi, aim);
    }
#pragma unroll
    for (int o = NCP; o < LT; o <<= 1) {
        are += __shfl_xor(are, o);
        aim += __shfl_xor(aim, o);
    }
    if (q != 0 || !live || c >= ncol || !set_active(a, s)) return;
#pragma unroll
    for (int part = 0; part < 2; ++part) {
        const int64_t row = 2 * k + part;
        const double v = a.scale * (part ? aim : are);
        if constexpr (EPI == EPI_ETA) {
            if (a.out_f32) ((float*)a.y)[row * a.ldy + s] = (float)v;
            else ((double*)a.y)[row * a.ldy + s] = v;
        } else {
            double* y = (double*)a.y + row * a.ldy + c;
            *y = a.accumulate ? *y + v : v;
        }
    }
}

// ------------------------------------------------------------- dispatch ----
template <int G, int NOPS, int MODE, int EPI>
static void launch_prec(const KArgs& k, int prec, dim3 grid, hipStream_t s) {
    switch (prec) {
        case CUT_F64: hipLaunchKernelGGL((k_pass<G, NOPS, CUT_F64, MODE, EPI>), grid, dim3(256), 0, s, k); break;
        case CUT_F32X: hipLaunchKernelGGL((k_pass<G, NOPS, CUT_F32X, MODE, EPI>), grid, dim3(256), 0, s, k); break;
        case CUT_F32C: hipLaunchKernelGGL((k_pass<G, NOPS, CUT_F32C, MODE, EPI>), grid, dim3(256), 0, s, k); break;
        default: hipLaunchKernelGGL((k_pass<G, NOPS, CUT_F32, MODE, EPI>), grid, dim3(256), 0, s, k); break;
    }
}

template <int G, int MODE, int EPI>
static void launch_nops(const KArgs& k, int prec, dim3 grid, hipStream_t s) {
    if constexpr (EPI == EPI_ETA) {
        hipLaunchKernelGGL((k_pass<G, 1, CUT_F64, MODE_BCAST, EPI_ETA>), grid, dim3(256), 0, s, k);
    } else {
        switch (k.nops) {
            case 1: launch_prec<G, 1, MODE, EPI>(k, prec, grid, s); break;
            case 2: launch_prec<G, 2, MODE, EPI>(k, prec, grid, s); break;
            case 3: launch_prec<G, 3, MODE, EPI>(k, prec, grid, s); break;
            case 4: launch_prec<G, 4, MODE, EPI>(k, prec, grid, s); break;
            case 5: launch_prec<G, 5, MODE, EPI>(k, prec, grid, s); break;
            case 6: launch_prec<G, 6, MODE, EPI>(k, prec, grid, s); break;
            case 7: launch_prec<G, 7, MODE, EPI>(k, prec, grid, s); break;
            default: launch_prec<G, 8, MODE, EPI>(k, prec, grid, s); break;
        }
    }
}

template <int MODE, int EPI>
static void launch_g(const KArgs& k, int prec, int G, dim3 grid, hipStream_t s) {
    switch (G) {
        case 1: launch_nops<1, MODE, EPI>(k, prec, grid, s); break;
        case 2: launch_nops<2, MODE, EPI>(k, prec, grid, s); break;
        case 4: launch_nops<4, MODE, EPI>(k, prec, grid, s); break;
        case 8: launch_nops<8, MODE, EPI>(k, prec, grid, s); break;
        case 16: launch_nops<16, MODE, EPI>(k, prec, grid, s); break;
        case 32: launch_nops<32, MODE, EPI>(k, prec, grid, s); break;
        default: launch_nops<64, MODE, EPI>(k, prec, grid, s); break;
    }
}

// lanes per record slot: the smallest power of two up to 64 holding nsets
static int group_width(int nsets) {
    int G = 1;
    while (G < nsets && G < 64) G <<= 1;
    return G;
}

// lane groups of a launch over the sets [s0, s1) of nsets: at least 8 lanes
// when the state has that many sets, since below 8 a lane group reads a whole
// cache line per operand for each set and gets no cheaper
static int range_group_width(const KArgs& k) {
    return group_width(std::max(k.s1 - k.s0, std::min(8, (int)k.nsets)));
}

// the kernels multiply row indices by 32-bit strides
static void check_ld(const PassArgs& p) {
    if (p.lda >= (int64_t)1 << 31 || p.ldb >= (int64_t)1 << 31 || p.ldy >= (int64_t)1 << 31)
        CUT_FAIL(CUT_E_INVAL, "leading dimension of 2^31 elements or more");
}

static KArgs make_kargs(const PassArgs& p) {
    const DevCSR& c = *p.csr;
    check_ld(p);
    KArgs k{};
    k.tasks = p.tasks ? p.tasks : c.tasks;
    k.ntasks = p.tasks ? p.ntasks : c.ntasks;
    k.per_xcd = p.tasks ? p.per_xcd : c.per_xcd;
    k.off = c.off;
    k.rec = c.rec;
    k.A = p.A;
    k.lda = p.lda;
    k.B = p.B;
    k.ldb = p.ldb;
    k.nsets = p.nsets;
    k.nops = p.nops;
    k.s0 = p.s1 > 0 ? p.s0 : 0;
    k.s1 = p.s1 > 0 ? p.s1 : p.nsets;
    k.nsteps = p.nsteps;
    k.step = p.step;
    k.y = p.y;
    k.ldy = p.ldy;
    k.accumulate = p.accumulate;
    k.out_f32 = p.precision != CUT_F64;
    k.scale = p.scale;
    k.stage = p.stage;
    k.ds = p.ds;
    k.z = p.z;
    k.acc = p.acc;
    k.xout = p.xout;
    k.hst = p.hst;
    k.ldh = p.ldh;
    const int64_t esz = p.precision == CUT_F64 ? 8 : 4;
    const int64_t ld = p.lda > p.ldb ? p.lda : p.ldb;
    const int64_t rows = c.rows > c.nseg ? c.rows : c.nseg;
    k.buf32 = (rows * ld * esz < (int64_t)0x7FFFFFFF) ? 1 : 0;
    return k;
}

// FP64 passes (and the generator pass, FP64 arithmetic) over a complex twin
// whose targets are all short: k_cshort
static bool cshort_usable(int mode, int epi, const PassArgs& p) {
    if (mode != MODE_BCAST || (epi != EPI_ETA && epi != EPI_Y) || p.csr->cx == nullptr || p.tasks != nullptr)
        return false;
    const DevCSR& c = *p.csr->cx;
    if (c.max_len > kShortMax || c.nrec == 0 || (int64_t)p.nops * p.nsets > 8) return false;
    if (epi == EPI_Y && p.precision != CUT_F64) return false;
    return 2 * c.na * p.lda * 8 < ((int64_t)1 << 32) && 2 * c.nb * p.ldb * 8 < ((int64_t)1 << 32);
}

template <int EPI, bool GPAIR>
static void launch_cshort_e(const KArgs& k, int ncp, int64_t nt, hipStream_t s) {
    const int tpw = 64 / (8 * ncp);
    const dim3 grid((unsigned)((nt + 4 * tpw - 1) / (4 * tpw)));
    switch (ncp) {
        case 1: hipLaunchKernelGGL((k_cshort<1, EPI, GPAIR>), grid, dim3(256), 0, s, k, nt); break;
        case 2: hipLaunchKernelGGL((k_cshort<2, EPI, GPAIR>), grid, dim3(256), 0, s, k, nt); break;
        case 4: hipLaunchKernelGGL((k_cshort<4, EPI, GPAIR>), grid, dim3(256), 0, s, k, nt); break;
        default: hipLaunchKernelGGL((k_cshort<8, EPI, GPAIR>), grid, dim3(256), 0, s, k, nt); break;
    }
}

static void launch_cshort(int epi, const PassArgs& p, hipStream_t s) {
    PassArgs r = p;
    r.csr = p.csr->cx;
    const int64_t nt = r.csr->nseg;
    if (nt == 0) return;
    const KArgs k = make_kargs(r);
    const int ncol = p.nops * p.nsets;
    const int ncp = ncol <= 1 ? 1 : ncol <= 2 ? 2 : ncol <= 4 ? 4 : 8;
    const bool gpair = p.lda == 1 && (reinterpret_cast<uintptr_t>(p.A) & 15) == 0;
    if (epi == EPI_ETA) {
        if (gpair) launch_cshort_e<EPI_ETA, true>(k, ncp, nt, s);
        else launch_cshort_e<EPI_ETA, false>(k, ncp, nt, s);
    } else {
        if (gpair) launch_cshort_e<EPI_Y, true>(k, ncp, nt, s);
        else launch_cshort_e<EPI_Y, false>(k, ncp, nt, s);
    }
}

static int cpass_columns(int ncol) {
    return ncol <= 1 ? 1 : ncol <= 2 ? 2 : ncol <= 4 ? 4 : ncol <= 8 ? 8 : ncol <= 16 ? 16 : 32;
}

// FP64 forward passes of a record set with a complex twin (Pauli-boson E_L
// and E_C) up to 32 columns run k_cpass; everything else the real-split form
static bool cpass_usable(int mode, int epi, const PassArgs& p) {
    if (mode != MODE_BCAST || (epi != EPI_Y && epi != EPI_RK) || p.csr->cx == nullptr ||
        p.precision != CUT_F64 || p.tasks != nullptr || (int64_t)p.nops * p.nsets > 32)
        return false;
    // 32-bit byte offsets into both operand arrays
    const DevCSR& c = *p.csr->cx;
    return 2 * c.na * p.lda * 8 < ((int64_t)1 << 32) && 2 * c.nb * p.ldb * 8 < ((int64_t)1 << 32);
}

template <int EPI, bool GPAIR>
static void launch_cpass_e(const KArgs& k, int ncp, dim3 grid, hipStream_t s) {
    switch (ncp) {
        case 1: hipLaunchKernelGGL((k_cpass<1, EPI, GPAIR>), grid, dim3(256), 0, s, k); break;
        case 2: hipLaunchKernelGGL((k_cpass<2, EPI, GPAIR>), grid, dim3(256), 0, s, k); break;
        case 4: hipLaunchKernelGGL((k_cpass<4, EPI, GPAIR>), grid, dim3(256), 0, s, k); break;
        case 8: hipLaunchKernelGGL((k_cpass<8, EPI, GPAIR>), grid, dim3(256), 0, s, k); break;
        case 16: hipLaunchKernelGGL((k_cpass<16, EPI, GPAIR>), grid, dim3(256), 0, s, k); break;
        default: hipLaunchKernelGGL((k_cpass<32, EPI, GPAIR>), grid, dim3(256), 0, s, k); break;
    }
}

static void launch_cpass(int epi, const PassArgs& p, hipStream_t s) {
    PassArgs r = p;
    r.csr = p.csr->cx;
    if (r.csr->nseg == 0) return;
    const KArgs k = make_kargs(r);
    if (k.ntasks == 0) return;
    const dim3 grid((unsigned)(k.per_xcd > 0 ? 8 * k.per_xcd : k.ntasks));
    const int ncp = cpass_columns(p.nops * p.nsets);
    const bool gpair = p.lda == 1 && (reinterpret_cast<uintptr_t>(p.A) & 15) == 0;
    // one set, an even column count and 16-byte aligned operand rows: two
    // columns per lane (measured on the five-mode benchmark: 4.09 ms for the
    // action with all outside-space records against 6.07 ms for one column
    // per lane and 4.46 ms for four)
    if (gpair && p.nsets == 1 && p.nops % 2 == 0 && ncp >= 2 && ncp <= 8 && p.ldb % 2 == 0 &&
        (reinterpret_cast<uintptr_t>(p.B) & 15) == 0) {
        const bool rk = epi == EPI_RK;
#define CUT_CPASSW(NCP_)                                                                           \
    if (rk) hipLaunchKernelGGL((k_cpassw<NCP_, EPI_RK, 2>), grid, dim3(256), 0, s, k);            \
    else hipLaunchKernelGGL((k_cpassw<NCP_, EPI_Y, 2>), grid, dim3(256), 0, s, k);
        if (ncp == 2) {
            CUT_CPASSW(2)
        } else if (ncp == 4) {
            CUT_CPASSW(4)
        } else {
            CUT_CPASSW(8)
        }
#undef CUT_CPASSW
        return;
    }
    if (epi == EPI_Y) {
        if (gpair) launch_cpass_e<EPI_Y, true>(k, ncp, grid, s);
        else launch_cpass_e<EPI_Y, false>(k, ncp, grid, s);
    } else {
        if (gpair) launch_cpass_e<EPI_RK, true>(k, ncp, grid, s);
        else launch_cpass_e<EPI_RK, false>(k, ncp, grid, s);
    }
}

void launch_pass(int mode, int epi, const PassArgs& p, hipStream_t s) {
    check_ld(p);
    if (cshort_usable(mode, epi, p)) {
        launch_cshort(epi, p, s);
        return;
    }
    if (cpass_usable(mode, epi, p)) {
        launch_cpass(epi, p, s);
        return;
    }
    if (p.csr->nseg == 0) return;
    const KArgs k = make_kargs(p);
    if (k.ntasks == 0) return;
    const int G = std::min(std::max(range_group_width(k), (int)p.gfloor), (int)p.gmax);
    const int64_t nblk = k.per_xcd > 0 ? 8 * k.per_xcd : k.ntasks;
    dim3 grid((unsigned)nblk, (unsigned)((k.s1 - k.s0 + G - 1) / G));
    if (mode == MODE_BCAST) {
        if (epi == EPI_Y) launch_g<MODE_BCAST, EPI_Y>(k, p.precision, G, grid, s);
        else if (epi == EPI_ETA) launch_g<MODE_BCAST, EPI_ETA>(k, p.precision, G, grid, s);
        else launch_g<MODE_BCAST, EPI_RK>(k, p.precision, G, grid, s);
    } else {
        launch_g<MODE_REDOPS, EPI_Y>(k, p.precision, G, grid, s);
    }
}

// ----------------------------------------------------- shared-triple tiles ----
// One workgroup per (tile tau, chunk of G sets).  The M member rows tau+w are
// staged in LDS as [M][NOPS+1][G] (operand columns, then the generator); each
// wavefront then walks members t = wave, wave+4, ...: every record of member t
// reads one operand from LDS and the other from its quadratic row (a small,
// L2-resident set), and the member's sum goes to its partial slot.
struct TileKArgs {
    const int32_t* rows;
    const uint8_t* slot;
    const uint2* rec;
    int32_t M, RT;
    const void* H;
    int64_t lde;
    const void* X;
    int64_t ldx;
    int32_t nsets;
    const int32_t* nsteps;
    const int32_t* step;
    double* P;
    int64_t ldp;
    int64_t pstride;
};

template <int G, int NOPS, int PREC>
__global__ __launch_bounds__(256) void k_tile(TileKArgs a) {
    using T = typename PrecT<PREC>::T;
    constexpr int R = 64 / G;
#ifndef CUT_TILE_UNROLL
#define CUT_TILE_UNROLL 4
#endif
    constexpr int U = (NOPS <= 2) ? 8 : CUT_TILE_UNROLL;
    constexpr int W = NOPS + 1;
    extern __shared__ __align__(16) unsigned char tile_lds[];
    T* lds = reinterpret_cast<T*>(tile_lds);
    const int64_t tile = blockIdx.x;
    const int s0 = blockIdx.y * G;
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int sg = lane % G, sub = lane / G;
    const int s = s0 + sg;
    const int nsets = a.nsets;
    const bool act = s < nsets && (a.nsteps == nullptr || a.nsteps[s] > *a.step);
    const int sl = s < nsets ? s : nsets - 1;
    const int M = a.M, RT = a.RT;
    const int32_t* trows = a.rows + tile * M;
    const T* __restrict__ H = (const T*)a.H;
    const T* __restrict__ X = (const T*)a.X;
    constexpr int per_row = W * G;
    for (int e = threadIdx.x; e < M * per_row; e += 256) {
        const int r = e / per_row, rem = e - r * per_row, c = rem / G, ss = rem - c * G;
        const int64_t grow = trows[r];
        const int sc = (s0 + ss < nsets) ? s0 + ss : nsets - 1;
        lds[e] = (c < NOPS) ? X[grow * a.ldx + (int64_t)c * nsets + sc] : H[grow * a.lde + sc];
    }
    __syncthreads();
    int coff[NOPS];
#pragma unroll
    for (int op = 0; op < NOPS; ++op) coff[op] = sl + op * nsets;
    for (int t = wave; t < M; t += 4) {
        const uint2* tr = a.rec + (tile * M + t) * (int64_t)RT;
        Acc<PREC> acc[NOPS];
        for (int r0 = 0; r0 < RT; r0 += R * U) {
            uint2 rr[U];
            bool ok[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int r = r0 + u * R + sub;
                ok[u] = r < RT;
                rr[u] = tr[ok[u] ? r : RT - 1];
            }
            T av[U];
            T bv[U][NOPS];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int64_t quad = rr[u].x;
                const T* lrow = lds + (int)((rr[u].y >> 1) & 0x7FFFu) * per_row + sg;
                if (rr[u].y & 1u) {  // generator from LDS, operand from the quadratic row
                    av[u] = lrow[NOPS * G];
                    const T* xr = X + quad * a.ldx;
#pragma unroll
                    for (int op = 0; op < NOPS; ++op) bv[u][op] = xr[coff[op]];
                } else {             // generator from the quadratic row, operand from LDS
                    av[u] = H[quad * a.lde + sl];
#pragma unroll
                    for (int op = 0; op < NOPS; ++op) bv[u][op] = lrow[op * G];
                }
            }
            decltype(left_term<PREC>(0.0, av[0])) tl[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const double cf = ok[u] ? (double)__builtin_bit_cast(float, rr[u].y & 0xFFFF0000u) : 0.0;
                tl[u] = left_term<PREC>(cf, av[u]);
            }
            add_group<PREC, U, NOPS>(acc, tl, bv);
        }
        double v[NOPS];
#pragma unroll
        for (int op = 0; op < NOPS; ++op) {
            v[op] = acc[op].get();
#pragma unroll
            for (int o = G; o < 64; o <<= 1) v[op] += __shfl_xor(v[op], o);
        }
        if (sub == 0 && act) {
            double* P = a.P + (int64_t)a.slot[tile * M + t] * a.pstride + (int64_t)trows[t] * a.ldp + s;
#pragma unroll
            for (int op = 0; op < NOPS; ++op) P[(int64_t)op * nsets] = v[op];
        }
    }
}

// Tile kernel for 64-set chunks (blockIdx.y): one workgroup of 8 wavefronts
// per tile, lane = set.  The M member rows are staged in LDS ([member][op
// columns, then eta][64 sets]) by wavefront-uniform 64-set runs through buffer
// loads; wavefront w then takes members w, w+8, ...  A member's RT records (a
// vector load of 64 at a time, handed out by readlane) come in two halves:
// first generator = quadratic row (one gather) with the operand from LDS, then
// generator from LDS with the operand = quadratic row (NOPS gathers); each
// batch of 4 records issues its gathers before any arithmetic.
template <int NOPS, int PREC>
__global__ __launch_bounds__(512) void k_tile64(TileKArgs a) {
    using T = typename PrecT<PREC>::T;
    constexpr int ROW = (NOPS + 1) * 64;
    constexpr int UA = 4;  // records per batch, first half (one gather each)
    constexpr int U = 4;   // records per batch, second half (NOPS gathers each)
    extern __shared__ __align__(16) unsigned char t64_lds[];
    T* lds = reinterpret_cast<T*>(t64_lds);  // [M][ROW]
    const int64_t tile = blockIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int nsets = a.nsets;
    const int s = (int)blockIdx.y * 64 + lane;
    const int sl = s < nsets ? s : nsets - 1;
    const bool act = s < nsets && (a.nsteps == nullptr || a.nsteps[s] > *a.step);
    const int M = a.M, RT = a.RT, half = RT / 2;
    const int32_t* trows = a.rows + tile * M;
    const auto rsH = row_rsrc(a.H, 0x7FFFFFFF);
    const auto rsX = row_rsrc(a.X, 0x7FFFFFFF);
    const int32_t lde_b = (int32_t)(a.lde * (int64_t)sizeof(T)), ldx_b = (int32_t)(a.ldx * (int64_t)sizeof(T));
    const uint32_t voff = (uint32_t)sl * (uint32_t)sizeof(T);
    // staging in batches of 16 runs per wavefront: all loads of a batch are in
    // flight before the first LDS store
    constexpr int SB = 16;
    const int nruns = M * (NOPS + 1);
    for (int q0 = wave; q0 < nruns; q0 += 8 * SB) {
        T v[SB];
#pragma unroll
        for (int k = 0; k < SB; ++k) {
            const int q = q0 + 8 * k;
            const int qc = q < nruns ? q : nruns - 1;
            const int mr = qc / (NOPS + 1), c = qc - mr * (NOPS + 1);
            const int32_t grow = __builtin_amdgcn_readfirstlane(trows[mr]);
            v[k] = c < NOPS ? buf_load<T>(rsX, voff, grow * ldx_b + c * nsets * (int32_t)sizeof(T))
                            : buf_load<T>(rsH, voff, grow * lde_b);
        }
#pragma unroll
        for (int k = 0; k < SB; ++k) {
            const int q = q0 + 8 * k;
            if (q < nruns) {
                const int mr = q / (NOPS + 1), c = q - mr * (NOPS + 1);
                lds[mr * ROW + c * 64 + lane] = v[k];
            }
        }
    }
    __syncthreads();
    for (int t = wave; t < M; t += 8) {
        const uint2* tr = a.rec + (tile * M + t) * (int64_t)RT;
        Acc<PREC> acc[NOPS];
        uint2 mine = tr[lane < RT ? lane : RT - 1];
        int base = 0;  // first record held in `mine`
        auto rec_at = [&](int r, uint32_t& x, uint32_t& y) {
            if (r - base >= 64) {
                base += 64;
                mine = tr[base + lane < RT ? base + lane : RT - 1];
            }
            x = (uint32_t)__builtin_amdgcn_readlane((int)mine.x, r - base);
            y = (uint32_t)__builtin_amdgcn_readlane((int)mine.y, r - base);
        };
        // first half: generator = quadratic row eta, operand from LDS
        for (int r0 = 0; r0 < half; r0 += UA) {
            uint32_t rx[UA], ry[UA];
            T gv[UA];
#pragma unroll
            for (int u = 0; u < UA; ++u) {
                rec_at(r0 + u < half ? r0 + u : half - 1, rx[u], ry[u]);
                gv[u] = buf_load<T>(rsH, voff, (int32_t)rx[u] * lde_b);
            }
            decltype(left_term<PREC>(0.0, gv[0])) tl[UA];
            T lv[UA][NOPS];
#pragma unroll
            for (int u = 0; u < UA; ++u) {
                const uint32_t fb = r0 + u < half ? (ry[u] & 0xFFFF0000u) : 0u;
                tl[u] = left_term<PREC>((double)__builtin_bit_cast(float, fb), gv[u]);
                const T* lrow = lds + (int)((ry[u] >> 1) & 0x7FFFu) * ROW + lane;
#pragma unroll
                for (int op = 0; op < NOPS; ++op) lv[u][op] = lrow[op * 64];
            }
            add_group<PREC, UA, NOPS>(acc, tl, lv);
        }
        // second half: generator from LDS, operand = quadratic row
        for (int r0 = half; r0 < RT; r0 += U) {
            uint32_t rx[U], ry[U];
            T bv[U][NOPS];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                rec_at(r0 + u < RT ? r0 + u : RT - 1, rx[u], ry[u]);
#pragma unroll
                for (int op = 0; op < NOPS; ++op)
                    bv[u][op] = buf_load<T>(rsX, voff, (int32_t)rx[u] * ldx_b + op * nsets * (int32_t)sizeof(T));
            }
            decltype(left_term<PREC>(0.0, bv[0][0])) tl[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const uint32_t fb = r0 + u < RT ? (ry[u] & 0xFFFF0000u) : 0u;
                const T* lrow = lds + (int)((ry[u] >> 1) & 0x7FFFu) * ROW + lane;
                tl[u] = left_term<PREC>((double)__builtin_bit_cast(float, fb), lrow[NOPS * 64]);
            }
            add_group<PREC, U, NOPS>(acc, tl, bv);
        }
        if (act) {
            double* P = a.P + (int64_t)a.slot[tile * M + t] * a.pstride + (int64_t)trows[t] * a.ldp + s;
#pragma unroll
            for (int op = 0; op < NOPS; ++op) P[(int64_t)op * nsets] = acc[op].get();
        }
    }
}

// Fixed-order sum of the 4 partial slots of rows [row0, row0 + nrows), then the
// epilogue (store / accumulate, or the RK stage update).
template <int NOPS, int PREC, int EPI>
__global__ __launch_bounds__(256) void k_combine(KArgs a, const double* __restrict__ P, int64_t pstride,
                                                 int64_t ldp, int64_t row0, int64_t nrows) {
    using T = typename PrecT<PREC>::T;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nrows * a.nsets) return;
    const int64_t row = row0 + q / a.nsets;
    const int s = (int)(q % a.nsets);
    if (a.nsteps && a.nsteps[s] <= *a.step) return;
    const double* p = P + row * ldp + s;
    double v[NOPS];
#pragma unroll
    for (int op = 0; op < NOPS; ++op) {
        const int64_t o = (int64_t)op * a.nsets;
        v[op] = ((__builtin_nontemporal_load(p + o) + __builtin_nontemporal_load(p + pstride + o)) +
                 __builtin_nontemporal_load(p + 2 * pstride + o)) +
                __builtin_nontemporal_load(p + 3 * pstride + o);
    }
    if constexpr (EPI == EPI_Y) {
        double* y = (double*)a.y + row * a.ldy + s;
#pragma unroll
        for (int op = 0; op < NOPS; ++op) {
            double& o = y[(int64_t)op * a.nsets];
            o = a.accumulate ? o + a.scale * v[op] : a.scale * v[op];
        }
    } else {
        rk_epilogue<NOPS, T>(a, row, s, v);
    }
}

// sets per tile workgroup: 64 (the 8-wavefront kernel) when the member rows of
// 64 sets fit in 64 KiB of LDS, else 32 or 16
static int tile_width(const Graph& g, int nsets, int nops, int prec) {
    if (nsets > 32 && (size_t)g.tiles.M * (nops + 1) * 64 * (prec == CUT_F64 ? 8 : 4) <= 65536) return 64;
    return nsets <= 16 ? 16 : 32;
}

// Long segments: the partial rows of their chunks [cstart[l], cstart[l+1])
// added in chunk order, then the epilogue on row crow[l].
template <int NOPS, int PREC, int EPI>
__global__ __launch_bounds__(256) void k_chunk_combine(KArgs a, const double* __restrict__ P, int64_t ldp,
                                                       const int64_t* __restrict__ cstart,
                                                       const int32_t* __restrict__ crow, int64_t nlong) {
    using T = typename PrecT<PREC>::T;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int nr = a.s1 - a.s0;
    if (q >= nlong * nr) return;
    const int64_t l = q / nr;
    const int s = a.s0 + (int)(q % nr);
    if (a.nsteps && a.nsteps[s] <= *a.step) return;
    const int64_t row = crow[l];
    double v[NOPS];
#pragma unroll
    for (int op = 0; op < NOPS; ++op) v[op] = 0.0;
    for (int64_t c = cstart[l]; c < cstart[l + 1]; ++c) {
        const double* p = P + c * ldp + s;
#pragma unroll
        for (int op = 0; op < NOPS; ++op) v[op] += __builtin_nontemporal_load(p + (int64_t)op * a.nsets);
    }
    if constexpr (EPI == EPI_Y) {
        double* y = (double*)a.y + row * a.ldy + s;
#pragma unroll
        for (int op = 0; op < NOPS; ++op) {
            double& o = y[(int64_t)op * a.nsets];
            o = a.accumulate ? o + a.scale * v[op] : a.scale * v[op];
        }
    } else {
        rk_epilogue<NOPS, T>(a, row, s, v);
    }
}

template <int NOPS, int EPI>
static void launch_chunk_combine_p(const KArgs& k, int prec, const ChunkPlan& c, const double* P, int64_t ldp,
                                   hipStream_t s) {
    const unsigned nb = (unsigned)((c.nlong * (k.s1 - k.s0) + 255) / 256);
    switch (prec) {
        case CUT_F64: hipLaunchKernelGGL((k_chunk_combine<NOPS, CUT_F64, EPI>), dim3(nb), dim3(256), 0, s, k, P, ldp, c.cstart, c.crow, c.nlong); break;
        case CUT_F32X: hipLaunchKernelGGL((k_chunk_combine<NOPS, CUT_F32X, EPI>), dim3(nb), dim3(256), 0, s, k, P, ldp, c.cstart, c.crow, c.nlong); break;
        case CUT_F32C: hipLaunchKernelGGL((k_chunk_combine<NOPS, CUT_F32C, EPI>), dim3(nb), dim3(256), 0, s, k, P, ldp, c.cstart, c.crow, c.nlong); break;
        default: hipLaunchKernelGGL((k_chunk_combine<NOPS, CUT_F32, EPI>), dim3(nb), dim3(256), 0, s, k, P, ldp, c.cstart, c.crow, c.nlong); break;
    }
}

template <int EPI>
static void launch_chunk_combine(const KArgs& k, int prec, const ChunkPlan& c, const double* P, int64_t ldp,
                                 hipStream_t s) {
    switch (k.nops) {
        case 1: launch_chunk_combine_p<1, EPI>(k, prec, c, P, ldp, s); break;
        case 2: launch_chunk_combine_p<2, EPI>(k, prec, c, P, ldp, s); break;
        case 3: launch_chunk_combine_p<3, EPI>(k, prec, c, P, ldp, s); break;
        case 4: launch_chunk_combine_p<4, EPI>(k, prec, c, P, ldp, s); break;
        case 5: launch_chunk_combine_p<5, EPI>(k, prec, c, P, ldp, s); break;
        case 6: launch_chunk_combine_p<6, EPI>(k, prec, c, P, ldp, s); break;
        case 7: launch_chunk_combine_p<7, EPI>(k, prec, c, P, ldp, s); break;
        default: launch_chunk_combine_p<8, EPI>(k, prec, c, P, ldp, s); break;
    }
}

size_t chunk_partial_bytes(const Graph& g, int32_t nsets, int32_t nops) {
    const ChunkPlan& c = g.csr[0][0].cp;
    size_t slots = c.nlong > 0 ? (size_t)c.nslots : 0;
    if (g.qb.active) slots = std::max(slots, (size_t)g.qb.cp.nslots);
    return slots * nops * nsets * sizeof(double);
}

static bool quad_and_tiles(const Graph& g, int32_t nsets, int32_t nops, int32_t precision);

size_t forward_partial_bytes(const Graph& g, int32_t nsets, int32_t nops, int32_t precision) {
    // the chunk plan's rows are always needed: a launch over part of the sets
    // runs the plain chunked form whatever the tiling
    const size_t chunk = chunk_partial_bytes(g, nsets, nops);
    if (tiles_usable(g, nsets, nops, precision)) {
        size_t b = tile_partial_bytes(g, nsets, nops);
        if (quad_and_tiles(g, nsets, nops, precision)) b += (size_t)g.qb.cp_lead.nslots * nops * nsets * sizeof(double);
        return std::max(b, chunk);
    }
    return chunk;
}

// ------------------------------------------------ quadratic-target blocks ----
// One workgroup (8 wavefronts) per (group pair, triple range), 64 coefficient
// sets per blockIdx.y.  Wavefront w owns mode u = g1 + w and the targets
// {u, v}, v = g2 + j (j < 8, u < v); lane = set.  Per triple T of the range (in
// lexicographic order) the rows T+w of the group modes are staged in LDS
// ([slot][op columns, then eta][64 sets]); wavefront w stages slots 2w, 2w+1
// (slot w on a diagonal pair) with one buffer load per 64-set run at a
// uniform row offset, loading the next triple's rows during the current
// triple's arithmetic and writing them to the other buffer.  Each live target
// adds its two records (T+u, T+v), (T+v, T+u) from LDS; the factors are the
// common magnitude with the sign bits of the plan.  Row indices and sign words
// of 64 consecutive triples are fetched with one vector load and handed out by
// readlane.  The sum of target j over the range is partial row tslot + r.
struct QBArgs {
    const int32_t* row4;
    const uint64_t* tmask;
    const int2* bpair;
    const uint32_t* sgn;
    const int32_t* tslot;
    float fmag;
    int32_t m, nr;
    int64_t ntrip;
    const void* A;
    int64_t lda;
    const void* B;
    int64_t ldb;
    int32_t nsets;
    const int32_t* nsteps;
    const int32_t* step;
    double* part;
    int64_t ldp;
};

template <int NOPS, int PREC>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void k_qblock(QBArgs a) {
    using T = typename PrecT<PREC>::T;
    // Compensated-float passes accumulate here the CUT_F32X way (exact
    // products and sums in FP64): as accurate or more than the compensated
    // float sum, and 2 VALU operations per term instead of 4.5 (a two-sum for
    // every two records); the operands and their staging stay float.
    constexpr int APREC = PREC == CUT_F32C ? CUT_F32X : PREC;
    constexpr int ROW = (NOPS + 1) * 64;   // staged elements per row
    extern __shared__ __align__(16) unsigned char qb_lds[];
    T* lds = reinterpret_cast<T*>(qb_lds);  // [2][16][ROW]
    const int bp = (int)(blockIdx.x / (unsigned)a.nr), r = (int)(blockIdx.x % (unsigned)a.nr);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63;
    const int nsets = a.nsets;
    const int s = (int)blockIdx.y * 64 + lane;
    const int sl = s < nsets ? s : nsets - 1;
    const int m = a.m;
    const int2 gp = a.bpair[bp];
    const bool diag = gp.x == gp.y;
    const int64_t t0 = (int64_t)r * a.ntrip / a.nr, t1 = (int64_t)(r + 1) * a.ntrip / a.nr;
    const int u = gp.x + wave;
    const auto rsA = row_rsrc(a.A, 0x7FFFFFFF);
    const auto rsB = row_rsrc(a.B, 0x7FFFFFFF);
    const int32_t lda_b = (int32_t)(a.lda * (int64_t)sizeof(T)), ldb_b = (int32_t)(a.ldb * (int64_t)sizeof(T));
    const uint32_t voff = (uint32_t)sl * (uint32_t)sizeof(T);
    // staging slots of this wavefront and their modes
    const int nmine = diag ? 1 : 2;
    int smode[2];
    int sslot[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        sslot[h] = diag ? wave : 2 * wave + h;
        smode[h] = sslot[h] < 8 ? gp.x + sslot[h] : gp.y + (sslot[h] - 8);
    }
    int32_t slot[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) slot[j] = __builtin_amdgcn_readfirstlane(a.tslot[bp * 64 + wave * 8 + j]);
    const float fpos = a.fmag;
    const uint32_t* sgw = a.sgn + ((int64_t)bp * 8 + wave) * a.ntrip;
    Acc<APREC> acc[8][NOPS];
    // per-window (64 triples) lane data: row of each staging slot, sign word
    int32_t rowv[2] = {-1, -1};
    uint32_t sgv = 0;
    auto window = [&](int64_t tw) {
        const int64_t ti = tw + lane;
        const bool in = ti < t1;
#pragma unroll
        for (int h = 0; h < 2; ++h)
            rowv[h] = (in && h < nmine && smode[h] < m) ? a.row4[ti * m + smode[h]] : -1;
        sgv = in ? sgw[ti] : 0u;
    };
    T nxt[2][NOPS + 1];
    auto load_rows = [&](int64_t ti) {
        const int li = (int)((ti - t0) & 63);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int32_t row = __builtin_amdgcn_readlane(rowv[h], li);
            if (h < nmine && row >= 0) {
#pragma unroll
                for (int c = 0; c < NOPS; ++c) nxt[h][c] = buf_load<T>(rsB, voff, row * ldb_b + c * nsets * (int32_t)sizeof(T));
                nxt[h][NOPS] = buf_load<T>(rsA, voff, row * lda_b);
            }
        }
    };
    auto store_rows = [&](int buf) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            if (h >= nmine) continue;
            T* dst = lds + (buf * 16 + sslot[h]) * ROW + lane;
#pragma unroll
            for (int c = 0; c <= NOPS; ++c) dst[c * 64] = nxt[h][c];
        }
    };
    if (t0 < t1) {
        window(t0);
        load_rows(t0);
        store_rows(0);
    }
    __syncthreads();
    for (int64_t ti = t0; ti < t1; ++ti) {
        const int buf = (int)((ti - t0) & 1);
        const int li = (int)((ti - t0) & 63);
        const uint32_t sbits = (uint32_t)__builtin_amdgcn_readlane((int)sgv, li);
        const bool more = ti + 1 < t1;
        if (more) {
            if (li == 63) window(ti + 1);
            load_rows(ti + 1);
        }
        const uint64_t tmk = a.tmask[ti];
        if (u < m && !((tmk >> u) & 1)) {
            const T* lu = lds + (buf * 16 + wave) * ROW + lane;
            const T eu = lu[NOPS * 64];
            T xu[NOPS];
#pragma unroll
            for (int op = 0; op < NOPS; ++op) xu[op] = lu[op * 64];
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const int v = gp.y + j;
                if (slot[j] < 0 || ((tmk >> v) & 1)) continue;
                const T* lv = lds + (buf * 16 + (diag ? j : 8 + j)) * ROW + lane;
                const T ev = lv[NOPS * 64];
                const float f1 = (sbits >> (2 * j)) & 1u ? -fpos : fpos;      // record (T+u, T+v)
                const float f2 = (sbits >> (2 * j + 1)) & 1u ? -fpos : fpos;  // record (T+v, T+u)
                const auto tu = left_term<APREC>((double)f1, eu);
                const auto tv = left_term<APREC>((double)f2, ev);
#pragma unroll
                for (int op = 0; op < NOPS; ++op) {
                    acc[j][op].add(tu, lv[op * 64]);
                    acc[j][op].add(tv, xu[op]);
                }
            }
        }
        if (more) store_rows(buf ^ 1);
        __syncthreads();
    }
    const bool act = s < nsets && (a.nsteps == nullptr || a.nsteps[s] > *a.step);
    if (!act) return;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if (slot[j] < 0) continue;
        double* P = a.part + (int64_t)(slot[j] + r) * a.ldp + s;
#pragma unroll
        for (int op = 0; op < NOPS; ++op) P[(int64_t)op * nsets] = acc[j][op].get();
    }
}

static size_t qblock_lds_bytes(int32_t nops, int32_t precision) {
    return (size_t)2 * 16 * (nops + 1) * 64 * (precision == CUT_F64 ? 8 : 4);
}

bool quadblocks_usable(const Graph& g, int32_t nsets, int32_t nops, int32_t precision) {
    (void)nsets;
    return g.qb.active && g.use_quadblocks && nops <= 5 && qblock_lds_bytes(nops, precision) <= 65536;
}

template <int NOPS>
static void launch_qblock_n(const QBArgs& q, int prec, dim3 grid, size_t lds, hipStream_t s) {
    switch (prec) {
        case CUT_F64: hipLaunchKernelGGL((k_qblock<NOPS, CUT_F64>), grid, dim3(512), lds, s, q); break;
        case CUT_F32X: hipLaunchKernelGGL((k_qblock<NOPS, CUT_F32X>), grid, dim3(512), lds, s, q); break;
        case CUT_F32C: hipLaunchKernelGGL((k_qblock<NOPS, CUT_F32C>), grid, dim3(512), lds, s, q); break;
        default: hipLaunchKernelGGL((k_qblock<NOPS, CUT_F32>), grid, dim3(512), lds, s, q); break;
    }
}

static void launch_qblock(const Graph& g, const PassArgs& a, double* partials, int64_t ldp, hipStream_t s) {
    const QuadBlockPlan& qp = g.qb;
    QBArgs q{};
    q.row4 = qp.row4;
    q.tmask = qp.tmask;
    q.bpair = qp.bpair;
    q.sgn = qp.sgn;
    q.tslot = qp.tslot;
    q.fmag = qp.fmag;
    q.m = qp.m;
    q.nr = qp.nr;
    q.ntrip = qp.ntrip;
    q.A = a.A;
    q.lda = a.lda;
    q.B = a.B;
    q.ldb = a.ldb;
    q.nsets = a.nsets;
    q.nsteps = a.nsteps;
    q.step = a.step;
    q.part = partials;
    q.ldp = ldp;
    dim3 grid((unsigned)(qp.nbp * qp.nr), (unsigned)((a.nsets + 63) / 64));
    const size_t lds = qblock_lds_bytes(a.nops, a.precision);
    switch (a.nops) {
        case 1: launch_qblock_n<1>(q, a.precision, grid, lds, s); break;
        case 2: launch_qblock_n<2>(q, a.precision, grid, lds, s); break;
        case 3: launch_qblock_n<3>(q, a.precision, grid, lds, s); break;
        case 4: launch_qblock_n<4>(q, a.precision, grid, lds, s); break;
        default: launch_qblock_n<5>(q, a.precision, grid, lds, s); break;
    }
}

// chunked forward pass: one launch whose first blocks sum long-segment chunks
// into partial rows and whose other blocks run the short segments with the
// epilogue; then the fixed-order combine of the partial rows with the epilogue
static void launch_chunked(const Graph& g, const ChunkPlan& c, int epi, const PassArgs& a, double* partials,
                           hipStream_t s, bool quad = false) {
    PassArgs r = a;
    r.tasks = c.short_tasks;
    r.ntasks = c.nshort;
    r.per_xcd = c.short_per_xcd;
    KArgs k = make_kargs(r);
    const int G = std::min(std::max(range_group_width(k), (int)a.gfloor), (int)a.gmax);
    const unsigned ychunks = (unsigned)((k.s1 - k.s0 + G - 1) / G);
    const int64_t ldp = (int64_t)a.nops * a.nsets;
    k.chunks = c.chunks;
    k.nchunks = c.nchunks;
    k.nchunk_blocks = c.chunks ? ((c.nchunks + 3) / 4 + 7) / 8 * 8 : 0;
    k.part = partials;
    k.ldp = ldp;
    const int64_t nshort_blocks = c.short_per_xcd > 0 ? 8 * c.short_per_xcd : c.nshort;
    if (k.nchunk_blocks + nshort_blocks > 0) {
        dim3 grid((unsigned)(k.nchunk_blocks + nshort_blocks), ychunks);
        if (epi == EPI_Y) launch_g<MODE_BCAST, EPI_Y>(k, a.precision, G, grid, s);
        else launch_g<MODE_BCAST, EPI_RK>(k, a.precision, G, grid, s);
    }
    if (quad) launch_qblock(g, a, partials, ldp, s);
    KArgs kc = make_kargs(a);
    if (epi == EPI_Y) launch_chunk_combine<EPI_Y>(kc, a.precision, c, partials, ldp, s);
    else launch_chunk_combine<EPI_RK>(kc, a.precision, c, partials, ldp, s);
}

static size_t tile_lds_bytes(const Graph& g, int32_t nsets, int32_t nops, int32_t prec) {
    return (size_t)g.tiles.M * (nops + 1) * tile_width(g, nsets, nops, prec) * (prec == CUT_F64 ? 8 : 4);
}

bool tiles_usable(const Graph& g, int32_t nsets, int32_t nops, int32_t precision) {
    return g.tiles.ok && g.use_tiles && nsets >= 8 &&
           (int64_t)tile_lds_bytes(g, nsets, nops, precision) <= g.max_lds;
}

// partial rows of the forward pass with quadratic-target blocks and tiles: the
// block plan's slots, then 4 tile slots per row
static bool quad_and_tiles(const Graph& g, int32_t nsets, int32_t nops, int32_t precision) {
    return quadblocks_usable(g, nsets, nops, precision) && g.qb.cp_lead.nlong > 0;
}

size_t tile_partial_bytes(const Graph& g, int32_t nsets, int32_t nops) {
    return (size_t)4 * g.N * nops * nsets * sizeof(double);
}

template <int G, int NOPS, int PREC>
static void launch_tile_k(const TileKArgs& t, dim3 grid, size_t lds, hipStream_t s) {
    hipLaunchKernelGGL((k_tile<G, NOPS, PREC>), grid, dim3(256), lds, s, t);
}

template <int NOPS, int PREC>
static void launch_tile_g(const TileKArgs& t, int G, dim3 grid, size_t lds, hipStream_t s) {
    if (G == 64) hipLaunchKernelGGL((k_tile64<NOPS, PREC>), grid, dim3(512), lds, s, t);
    else if (G == 16) launch_tile_k<16, NOPS, PREC>(t, grid, lds, s);
    else launch_tile_k<32, NOPS, PREC>(t, grid, lds, s);
}

template <int NOPS>
static void launch_tile_p(const TileKArgs& t, int prec, int G, dim3 grid, size_t lds, hipStream_t s) {
    switch (prec) {
        case CUT_F64: launch_tile_g<NOPS, CUT_F64>(t, G, grid, lds, s); break;
        case CUT_F32X: launch_tile_g<NOPS, CUT_F32X>(t, G, grid, lds, s); break;
        case CUT_F32C: launch_tile_g<NOPS, CUT_F32C>(t, G, grid, lds, s); break;
        default: launch_tile_g<NOPS, CUT_F32>(t, G, grid, lds, s); break;
    }
}

template <int NOPS, int EPI>
static void launch_combine_p(const KArgs& k, int prec, const double* P, int64_t pstride, int64_t ldp, int64_t row0,
                             int64_t nrows, hipStream_t s) {
    const unsigned nb = (unsigned)((nrows * k.nsets + 255) / 256);
    switch (prec) {
        case CUT_F64: hipLaunchKernelGGL((k_combine<NOPS, CUT_F64, EPI>), dim3(nb), dim3(256), 0, s, k, P, pstride, ldp, row0, nrows); break;
        case CUT_F32X: hipLaunchKernelGGL((k_combine<NOPS, CUT_F32X, EPI>), dim3(nb), dim3(256), 0, s, k, P, pstride, ldp, row0, nrows); break;
        case CUT_F32C: hipLaunchKernelGGL((k_combine<NOPS, CUT_F32C, EPI>), dim3(nb), dim3(256), 0, s, k, P, pstride, ldp, row0, nrows); break;
        default: hipLaunchKernelGGL((k_combine<NOPS, CUT_F32, EPI>), dim3(nb), dim3(256), 0, s, k, P, pstride, ldp, row0, nrows); break;
    }
}

template <int NOPS>
static void launch_tiles_nops(const TileKArgs& t, const KArgs& k, int epi, int prec, int G, dim3 grid, size_t lds,
                              int64_t row0, int64_t nrows, hipStream_t s) {
    launch_tile_p<NOPS>(t, prec, G, grid, lds, s);
    if (epi == EPI_Y) launch_combine_p<NOPS, EPI_Y>(k, prec, t.P, t.pstride, t.ldp, row0, nrows, s);
    else launch_combine_p<NOPS, EPI_RK>(k, prec, t.P, t.pstride, t.ldp, row0, nrows, s);
}

// whether launch_forward honours a set range [s0, s1) of `a`: a launch over a
// proper range of the sets runs the segment kernel over the plain chunk plan
// (always built with the tiling), as does a full-width launch with `narrow`;
// the block and tile kernels run only other full-width launches; the
// complex-record kernels always cover every set
bool forward_set_ranges(const Graph& g, const PassArgs& a) {
    (void)g;
    return !cpass_usable(MODE_BCAST, EPI_RK, a) && !cshort_usable(MODE_BCAST, EPI_RK, a);
}

void launch_forward(const Graph& g, int epi, const PassArgs& a_in, double* partials, hipStream_t s) {
    check_ld(a_in);
    PassArgs a = a_in;
    a.gmax = 64 >> g.bchunk;  // the tiling's B-chunk
    if (epi == EPI_ETA || a.csr != &g.csr[0][0] || partials == nullptr || cpass_usable(MODE_BCAST, epi, a) ||
        cshort_usable(MODE_BCAST, epi, a)) {
        launch_pass(MODE_BCAST, epi, a, s);
        return;
    }
    const bool ranged = a.narrow || (a.s1 > 0 && (a.s0 != 0 || a.s1 != a.nsets));
    if (ranged) {
        if (g.csr[0][0].cp.nlong > 0) launch_chunked(g, g.csr[0][0].cp, epi, a, partials, s);
        else launch_pass(MODE_BCAST, epi, a, s);
        return;
    }
    if (!tiles_usable(g, a.nsets, a.nops, a.precision)) {
        if (quadblocks_usable(g, a.nsets, a.nops, a.precision)) launch_chunked(g, g.qb.cp, epi, a, partials, s, true);
        else if (g.csr[0][0].cp.nlong > 0) launch_chunked(g, g.csr[0][0].cp, epi, a, partials, s);
        else launch_pass(MODE_BCAST, epi, a, s);
        return;
    }
    const TilePlan& tp = g.tiles;
    const int64_t ldp = (int64_t)a.nops * a.nsets;
    double* tpart = partials;
    if (quad_and_tiles(g, a.nsets, a.nops, a.precision)) {
        // quadratic targets: leading records (chunks) + blocks, own partial rows
        launch_chunked(g, g.qb.cp_lead, epi, a, partials, s, true);
        tpart = partials + g.qb.cp_lead.nslots * ldp;
    } else {
        // quadratic targets (all their records) through the segment kernel
        PassArgs r = a;
        r.tasks = tp.res_tasks;
        r.ntasks = tp.nres_tasks;
        r.per_xcd = tp.res_per_xcd;
        if (tp.nres_tasks > 0) launch_pass(MODE_BCAST, epi, r, s);
    }
    // quartic targets: tiles into partial slots, then the fixed-order combine
    const int G = tile_width(g, a.nsets, a.nops, a.precision);
    TileKArgs t{};
    t.rows = tp.rows;
    t.slot = tp.slot;
    t.rec = tp.rec;
    t.M = tp.M;
    t.RT = tp.RT;
    t.H = a.A;
    t.lde = a.lda;
    t.X = a.B;
    t.ldx = a.ldb;
    t.nsets = a.nsets;
    t.nsteps = a.nsteps;
    t.step = a.step;
    t.P = tpart;
    t.ldp = ldp;
    t.pstride = g.N * t.ldp;
    const KArgs k = make_kargs(a);
    dim3 grid((unsigned)tp.ntiles, (unsigned)((a.nsets + G - 1) / G));
    const size_t lds = tile_lds_bytes(g, a.nsets, a.nops, a.precision);
    const int64_t row0 = tp.nres, nrows = g.N - tp.nres;
    switch (a.nops) {
        case 1: launch_tiles_nops<1>(t, k, epi, a.precision, G, grid, lds, row0, nrows, s); break;
        case 2: launch_tiles_nops<2>(t, k, epi, a.precision, G, grid, lds, row0, nrows, s); break;
        case 3: launch_tiles_nops<3>(t, k, epi, a.precision, G, grid, lds, row0, nrows, s); break;
        case 4: launch_tiles_nops<4>(t, k, epi, a.precision, G, grid, lds, row0, nrows, s); break;
        case 5: launch_tiles_nops<5>(t, k, epi, a.precision, G, grid, lds, row0, nrows, s); break;
        case 6: launch_tiles_nops<6>(t, k, epi, a.precision, G, grid, lds, row0, nrows, s); break;
        case 7: launch_tiles_nops<7>(t, k, epi, a.precision, G, grid, lds, row0, nrows, s); break;
        default: launch_tiles_nops<8>(t, k, epi, a.precision, G, grid, lds, row0, nrows, s); break;
    }
}

// ------------------------------------------------------------ generator ----
// G2: eta_S = s_g * sum_t c_t eps_{a_t} h_{p_t} / (sum_t (c_t eps_{a_t})^2 + delta^2)
// over the stencil rows t of S (the generator records whose left input is a
// pair coordinate P_a); FP64 arithmetic, eta stored in the stage precision.
__global__ void k_g2(int64_t N, int32_t nsets, const int4* __restrict__ st,
                     const int32_t* __restrict__ pairs, const double* __restrict__ ftab,
                     double gsign, double d2, const double* __restrict__ h, int64_t ldh, void* eta,
                     int64_t lde, int eta_f32, const int32_t* nsteps, const int32_t* step) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t S = gid / nsets;
    const int s = (int)(gid % nsets);
    if (S >= N) return;
    if (nsteps && nsteps[s] <= *step) return;
    // all four stencil entries and their loads are issued before any use; an
    // unused entry (x < 0, always after the used ones; its y and z are 0)
    // reads row S and pair 0 and weighs zero, which leaves the sums exact
    int4 e[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) e[t] = st[S * 4 + t];
    double c[4], eps[4], hp[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const bool ok = e[t].x >= 0;
        c[t] = ok ? ftab[e[t].z] : 0.0;
        eps[t] = h[(int64_t)pairs[e[t].y] * ldh + s];
        hp[t] = h[(ok ? (int64_t)e[t].x : S) * ldh + s];
    }
    double num = 0.0, q = 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        num = __builtin_fma(c[t] * eps[t], hp[t], num);
        q = __builtin_fma(c[t] * eps[t], c[t] * eps[t], q);
    }
    const double v = e[0].x >= 0 ? gsign * num / (q + d2) : 0.0;
    if (eta_f32) ((float*)eta)[S * lde + s] = (float)v;
    else ((double*)eta)[S * lde + s] = v;
}

// VJP stage 1: per stencil target S, w_S = gbar_S / Q_S and u_S = gbar_S * Nsig_S / Q_S^2
// where Nsig_S = s_g * sum_t c_t eps h_p (so eta_S = Nsig_S / Q_S).
__global__ void k_g2_vjp_prep(int64_t N, int32_t nsets, const int4* __restrict__ st,
                              const int32_t* __restrict__ pairs, const double* __restrict__ ftab,
                              double gsign, double d2, const double* __restrict__ h, int64_t ldh,
                              const double* __restrict__ gbar, int64_t ldg, double* w, double* u) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t S = gid / nsets;
    const int s = (int)(gid % nsets);
    if (S >= N) return;
    double num = 0.0, q = 0.0;
    for (int t = 0; t < 4; ++t) {
        const int4 e = st[S * 4 + t];
        if (e.x < 0) break;
        const double c = ftab[e.z];
        const double eps = h[(int64_t)pairs[e.y] * ldh + s];
        num = __builtin_fma(c * eps, h[(int64_t)e.x * ldh + s], num);
        q = __builtin_fma(c * eps, c * eps, q);
    }
    const bool has = st[S * 4].x >= 0;
    q += d2;
    const double gb = has ? gbar[S * ldg + s] : 0.0;
    w[S * nsets + s] = gb / q;
    u[S * nsets + s] = gb * (gsign * num) / (q * q);
}

// VJP stage 2 (gather form, fixed order):
//  g_h[r] += sum_{(S,t): p_t(S)=r} s_g c_t eps_{a_t} w_S                    (d eta_S / d h_p)
//  g_h[P_a] += sum_{(S,t): a_t=a} (s_g c_t h_{p_t} w_S - 2 c_t^2 eps_a u_S)  (d eta_S / d eps_a)
__global__ void k_g2_vjp_partner(int64_t N, int32_t nsets, const int64_t* __restrict__ toff,
                                 const int4* __restrict__ tent, const int32_t* __restrict__ pairs,
                                 const double* __restrict__ ftab, double gsign,
                                 const double* __restrict__ h, int64_t ldh,
                                 const double* __restrict__ w, double* g_h, int64_t ldgh) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t r = gid / nsets;
    const int s = (int)(gid % nsets);
    if (r >= N) return;
    double acc = 0.0;
    for (int64_t q = toff[r]; q < toff[r + 1]; ++q) {
        const int4 e = tent[q];
        const double eps = h[(int64_t)pairs[e.y] * ldh + s];
        acc = __builtin_fma(gsign * ftab[e.z] * eps, w[(int64_t)e.x * nsets + s], acc);
    }
    g_h[r * ldgh + s] += acc;
}

// one wavefront per (pair a, set s); lanes stride over the pair's list
__global__ void k_g2_vjp_pairs(int64_t npairs, int32_t nsets, const int64_t* __restrict__ poff,
                               const int4* __restrict__ pent, const int32_t* __restrict__ pairs,
                               const double* __restrict__ ftab, double gsign,
                               const double* __restrict__ h, int64_t ldh,
                               const double* __restrict__ w, const double* __restrict__ u,
                               double* g_h, int64_t ldgh) {
    const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t a = wid / nsets;
    const int s = (int)(wid % nsets);
    if (a >= npairs) return;
    const int64_t pa = pairs[a];
    const double eps = h[pa * ldh + s];
    double acc = 0.0;
    for (int64_t q = poff[a] + lane; q < poff[a + 1]; q += 64) {
        const int4 e = pent[q];
        const double c = ftab[e.z];
        acc += gsign * c * h[(int64_t)e.y * ldh + s] * w[(int64_t)e.x * nsets + s] -
               2.0 * c * c * eps * u[(int64_t)e.x * nsets + s];
    }
    for (int o = 1; o < 64; o <<= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) g_h[pa * ldgh + s] += acc;
}

// G2 directional derivative along dh (quotient rule), FP64:
//   d eta_S = s_g (dnum Q - num dQ) / Q^2,  num = sum_t c_t eps_t h_{p_t},
//   dnum = sum_t c_t (d eps_t h_{p_t} + eps_t dh_{p_t}),  dQ = 2 sum_t c_t^2 eps_t d eps_t
__global__ void k_g2_jvp(int64_t N, int32_t nsets, const int4* __restrict__ st,
                         const int32_t* __restrict__ pairs, const double* __restrict__ ftab, double gsign,
                         double d2, const double* __restrict__ h, int64_t ldh, const double* __restrict__ dh,
                         int64_t lddh, double* deta, int64_t ldde) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t S = gid / nsets;
    const int s = (int)(gid % nsets);
    if (S >= N) return;
    double num = 0.0, q = 0.0, dnum = 0.0, dq = 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const int4 e = st[S * 4 + t];
        if (e.x < 0) break;
        const double c = ftab[e.z];
        const int64_t pa = pairs[e.y];
        const double eps = h[pa * ldh + s], deps = dh[pa * lddh + s];
        const double hp = h[(int64_t)e.x * ldh + s], dhp = dh[(int64_t)e.x * lddh + s];
        num = __builtin_fma(c * eps, hp, num);
        dnum = __builtin_fma(c * deps, hp, __builtin_fma(c * eps, dhp, dnum));
        q = __builtin_fma(c * eps, c * eps, q);
        dq = __builtin_fma(2.0 * c * c * eps, deps, dq);
    }
    const bool has = st[S * 4].x >= 0;
    q += d2;
    deta[S * ldde + s] = has ? gsign * (dnum * q - num * dq) / (q * q) : 0.0;
}

void launch_g2_jvp(const Graph& g, double delta, int32_t nsets, const double* h, int64_t ldh,
                   const double* dh, int64_t lddh, double* deta, int64_t ldde, hipStream_t s) {
    const int64_t n = g.N * nsets;
    hipLaunchKernelGGL(k_g2_jvp, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g.N, nsets, g.stencil,
                       g.pairs, g.ftab, g.gen_sign, delta * delta, h, ldh, dh, lddh, deta, ldde);
}

void launch_g2(const Graph& g, double delta, int32_t nsets, const double* h, int64_t ldh, void* eta,
               int64_t lde, bool eta_f32, const int32_t* nsteps, const int32_t* step, hipStream_t s) {
    const int64_t n = g.N * nsets;
    hipLaunchKernelGGL(k_g2, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g.N, nsets, g.stencil,
                       g.pairs, g.ftab, g.gen_sign, delta * delta, h, ldh, eta, lde, (int)eta_f32,
                       nsteps, step);
}

void launch_g2_vjp(const Graph& g, double delta, int32_t nsets, const double* h, int64_t ldh,
                   const double* gbar, int64_t ldg, double* g_h, int64_t ldgh, double* tmp,
                   hipStream_t s) {
    const int64_t n = g.N * nsets;
    double* w = tmp;
    double* u = tmp + n;
    const unsigned nb = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(k_g2_vjp_prep, dim3(nb), dim3(256), 0, s, g.N, nsets, g.stencil, g.pairs, g.ftab,
                       g.gen_sign, delta * delta, h, ldh, gbar, ldg, w, u);
    hipLaunchKernelGGL(k_g2_vjp_partner, dim3(nb), dim3(256), 0, s, g.N, nsets, g.st_t_off, g.st_t,
                       g.pairs, g.ftab, g.gen_sign, h, ldh, w, g_h, ldgh);
    const int64_t waves = g.npairs * nsets;
    hipLaunchKernelGGL(k_g2_vjp_pairs, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, g.npairs,
                       nsets, g.st_p_off, g.st_p, g.pairs, g.ftab, g.gen_sign, h, ldh, w, u, g_h, ldgh);
}

// ------------------------------------------------------------------- G1 ----
// Literal White-type generator from the diagonal pair energies:
//   eta_S = h_S / D_S,  D_S = 2 sum_{a in F(S)} |eps_a| + delta,  eps_a = h_{P_a},
// over the flipped pairs F(S) of an off-diagonal string S (its stencil entries'
// pairs); eta = 0 on block-diagonal strings.  FP64 arithmetic.
__device__ inline double g1_denominator(const int4* __restrict__ st, const int32_t* __restrict__ pairs,
                                        const double* __restrict__ h, int64_t ldh, int64_t S, int s,
                                        double delta, bool& has) {
    int4 e[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) e[t] = st[S * 4 + t];
    double d = 0.0;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
        const double eps = h[(int64_t)pairs[e[t].y] * ldh + s];
        d += e[t].x >= 0 ? 2.0 * __builtin_fabs(eps) : 0.0;
    }
    has = e[0].x >= 0;
    return d + delta;
}

__global__ void k_g1(int64_t N, int32_t nsets, const int4* __restrict__ st, const int32_t* __restrict__ pairs,
                     double delta, const double* __restrict__ h, int64_t ldh, void* eta, int64_t lde, int eta_f32,
                     const int32_t* nsteps, const int32_t* step) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t S = gid / nsets;
    const int s = (int)(gid % nsets);
    if (S >= N) return;
    if (nsteps && nsteps[s] <= *step) return;
    bool has;
    const double d = g1_denominator(st, pairs, h, ldh, S, s, delta, has);
    const double v = has ? h[S * ldh + s] / d : 0.0;
    if (eta_f32) ((float*)eta)[S * lde + s] = (float)v;
    else ((double*)eta)[S * lde + s] = v;
}

// d eta_S = dh_S / D_S - h_S dD_S / D_S^2,  dD_S = 2 sum_{a in F(S)} sign(eps_a) d eps_a
__global__ void k_g1_jvp(int64_t N, int32_t nsets, const int4* __restrict__ st, const int32_t* __restrict__ pairs,
                         double delta, const double* __restrict__ h, int64_t ldh, const double* __restrict__ dh,
                         int64_t lddh, double* deta, int64_t ldde) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t S = gid / nsets;
    const int s = (int)(gid % nsets);
    if (S >= N) return;
    double d = delta, dd = 0.0;
    for (int t = 0; t < 4; ++t) {
        const int4 e = st[S * 4 + t];
        if (e.x < 0) break;
        const int64_t pa = pairs[e.y];
        const double eps = h[pa * ldh + s];
        d += 2.0 * __builtin_fabs(eps);
        dd += 2.0 * (eps > 0.0 ? 1.0 : eps < 0.0 ? -1.0 : 0.0) * dh[pa * lddh + s];
    }
    const bool has = st[S * 4].x >= 0;
    deta[S * ldde + s] = has ? (dh[S * lddh + s] * d - h[S * ldh + s] * dd) / (d * d) : 0.0;
}

// VJP stage 1: w_S = gbar_S / D_S (added into g_h[S]) and u_S = gbar_S h_S / D_S^2
__global__ void k_g1_vjp_prep(int64_t N, int32_t nsets, const int4* __restrict__ st,
                              const int32_t* __restrict__ pairs, double delta, const double* __restrict__ h,
                              int64_t ldh, const double* __restrict__ gbar, int64_t ldg, double* u, double* g_h,
                              int64_t ldgh) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t S = gid / nsets;
    const int s = (int)(gid % nsets);
    if (S >= N) return;
    bool has;
    const double d = g1_denominator(st, pairs, h, ldh, S, s, delta, has);
    const double gb = has ? gbar[S * ldg + s] : 0.0;
    g_h[S * ldgh + s] += gb / d;
    u[S * nsets + s] = gb * h[S * ldh + s] / (d * d);
}

// VJP stage 2: g_h[P_a] -= 2 sign(eps_a) sum_{S: a in F(S)} u_S (one wavefront
// per (pair a, set s) over the pair's list of strings, fixed order)
__global__ void k_g1_vjp_pairs(int64_t npairs, int32_t nsets, const int64_t* __restrict__ poff,
                               const int4* __restrict__ pent, const int32_t* __restrict__ pairs,
                               const double* __restrict__ h, int64_t ldh, const double* __restrict__ u,
                               double* g_h, int64_t ldgh) {
    const int64_t wid = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    const int64_t a = wid / nsets;
    const int s = (int)(wid % nsets);
    if (a >= npairs) return;
    const int64_t pa = pairs[a];
    const double eps = h[pa * ldh + s];
    double acc = 0.0;
    for (int64_t q = poff[a] + lane; q < poff[a + 1]; q += 64) acc += u[(int64_t)pent[q].x * nsets + s];
    for (int o = 1; o < 64; o <<= 1) acc += __shfl_xor(acc, o);
    if (lane == 0) g_h[pa * ldgh + s] -= 2.0 * (eps > 0.0 ? 1.0 : eps < 0.0 ? -1.0 : 0.0) * acc;
}

void launch_g1(const Graph& g, double delta, int32_t nsets, const double* h, int64_t ldh, void* eta,
               int64_t lde, bool eta_f32, const int32_t* nsteps, const int32_t* step, hipStream_t s) {
    const int64_t n = g.N * nsets;
    hipLaunchKernelGGL(k_g1, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g.N, nsets, g.stencil, g.pairs,
                       delta, h, ldh, eta, lde, (int)eta_f32, nsteps, step);
}

void launch_g1_jvp(const Graph& g, double delta, int32_t nsets, const double* h, int64_t ldh,
                   const double* dh, int64_t lddh, double* deta, int64_t ldde, hipStream_t s) {
    const int64_t n = g.N * nsets;
    hipLaunchKernelGGL(k_g1_jvp, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g.N, nsets, g.stencil,
                       g.pairs, delta, h, ldh, dh, lddh, deta, ldde);
}

void launch_g1_vjp(const Graph& g, double delta, int32_t nsets, const double* h, int64_t ldh,
                   const double* gbar, int64_t ldg, double* g_h, int64_t ldgh, double* tmp, hipStream_t s) {
    const int64_t n = g.N * nsets;
    hipLaunchKernelGGL(k_g1_vjp_prep, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, g.N, nsets, g.stencil,
                       g.pairs, delta, h, ldh, gbar, ldg, tmp, g_h, ldgh);
    const int64_t waves = g.npairs * nsets;
    hipLaunchKernelGGL(k_g1_vjp_pairs, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, g.npairs, nsets,
                       g.st_p_off, g.st_p, g.pairs, h, ldh, tmp, g_h, ldgh);
}

// ---------------------------------------------------------- elementwise ----
__global__ void k_prep_state(const double* z, int64_t rows, int32_t nops, int32_t nsets, void* xsh,
                             int f32, double* hst) {
    const int64_t cols = (int64_t)nops * nsets;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= rows * cols) return;
    const double v = z[q];
    if (f32) ((float*)xsh)[q] = (float)v;
    else ((double*)xsh)[q] = v;
    const int64_t r = q / cols, c = q % cols;
    if (c < nsets) hst[r * nsets + c] = v;
}

void launch_prep_state(const double* z, int64_t rows, int32_t nops, int32_t nsets, void* xsh, bool f32,
                       double* hst, hipStream_t s) {
    const int64_t n = rows * nops * nsets;
    hipLaunchKernelGGL(k_prep_state, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, z, rows, nops,
                       nsets, xsh, (int)f32, hst);
}

// dst[r][c] = float(src[r][c]) (round to nearest even) for r < rows, c < cols
__global__ void k_round_f32(const double* __restrict__ src, int64_t lds, int64_t rows, int64_t cols,
                            float* __restrict__ dst, int64_t ldd) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= rows * cols) return;
    const int64_t r = q / cols, c = q % cols;
    dst[r * ldd + c] = (float)src[r * lds + c];
}

void launch_round_f32(const double* src, int64_t lds, int64_t rows, int64_t cols, float* dst, int64_t ldd,
                      hipStream_t s) {
    const int64_t n = rows * cols;
    if (n == 0) return;
    hipLaunchKernelGGL(k_round_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, lds, rows, cols,
                       dst, ldd);
}

// dst[r][c] = 0 for r < rows, c < cols (a kernel, not a memset, so that the
// clear can sit inside a captured graph)
__global__ void k_zero2d(double* dst, int64_t ld, int64_t rows, int64_t cols) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= rows * cols) return;
    dst[(q / cols) * ld + q % cols] = 0.0;
}

void launch_zero2d(double* dst, int64_t ld, int64_t rows, int64_t cols, hipStream_t s) {
    const int64_t n = rows * cols;
    if (n == 0) return;
    hipLaunchKernelGGL(k_zero2d, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, dst, ld, rows, cols);
}

// Column sums of squares of y [rows][cols] (contiguous rows), deterministic in
// two kernels.  k_colsq_partial: block (bx, by) owns the CB = min(cols, 256)
// columns from bx*CB; its threads are R = 256 / CB row lanes x CB columns, so
// every load instruction reads consecutive elements.  Row lane l of block by
// sums the rows by*R + l + k*R*gridDim.y (k = 0, 1, ...) into four running sums
// by k mod 4, added as (s0 + s1) + (s2 + s3); the row lanes are then added in
// order -> part[by][c].  k_colsq_finish adds the partial rows of a column in a
// fixed tree, scales by `weight` and accumulates into out[c] for the columns
// of active sets.
__global__ __launch_bounds__(256) void k_colsq_partial(const double* __restrict__ y, int64_t rows, int64_t cols,
                                                       double* __restrict__ part) {
    __shared__ double red[256];
    const int t = threadIdx.x;
    const int CB = cols < 256 ? (int)cols : 256;
    const int R = 256 / CB;
    const int rl = t / CB;
    const int64_t c = (int64_t)blockIdx.x * CB + t % CB;
    double acc = 0.0;
    if (rl < R && c < cols) {
        const int64_t step = (int64_t)R * gridDim.y;
        int64_t r = (int64_t)blockIdx.y * R + rl;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
        for (; r + 3 * step < rows; r += 4 * step) {
            const double v0 = y[r * cols + c], v1 = y[(r + step) * cols + c];
            const double v2 = y[(r + 2 * step) * cols + c], v3 = y[(r + 3 * step) * cols + c];
            s0 = __builtin_fma(v0, v0, s0);
            s1 = __builtin_fma(v1, v1, s1);
            s2 = __builtin_fma(v2, v2, s2);
            s3 = __builtin_fma(v3, v3, s3);
        }
        for (; r < rows; r += step) {
            const double v = y[r * cols + c];
            s0 = __builtin_fma(v, v, s0);
        }
        acc = (s0 + s1) + (s2 + s3);
    }
    red[t] = acc;
    __syncthreads();
    if (t < CB && c < cols) {
        double sum = 0.0;
        for (int l = 0; l < R; ++l) sum += red[l * CB + t];
        part[(int64_t)blockIdx.y * cols + c] = sum;
    }
}

__global__ __launch_bounds__(256) void k_colsq_finish(const double* __restrict__ part, int32_t nparts, int64_t cols,
                                                      int32_t nsets, const int32_t* nsteps, const int32_t* step,
                                                      double weight, double* out) {
    // one workgroup per column: thread t adds the partial rows t, t + 256, ...
    // in order, then a fixed pairwise tree over the 256 threads
    __shared__ double red[256];
    const int64_t c = blockIdx.x;
    const int t = threadIdx.x;
    double acc = 0.0;
    for (int b = t; b < nparts; b += 256) acc += part[(int64_t)b * cols + c];
    red[t] = acc;
    __syncthreads();
#pragma unroll
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) red[t] += red[t + w];
        __syncthreads();
    }
    if (t != 0) return;
    if (nsteps && nsteps[c % nsets] <= *step) return;
    out[c] += weight * red[0];
}

void launch_colsq_accumulate(const double* y, int64_t rows, int64_t cols, int32_t nsets, double* part,
                             int32_t nparts, const int32_t* nsteps, const int32_t* step, double weight,
                             double* out, hipStream_t s) {
    const int64_t cb = cols < 256 ? cols : 256;
    hipLaunchKernelGGL(k_colsq_partial, dim3((unsigned)((cols + cb - 1) / cb), (unsigned)nparts), dim3(256), 0, s, y,
                       rows, cols, part);
    hipLaunchKernelGGL(k_colsq_finish, dim3((unsigned)cols), dim3(256), 0, s, part, nparts, cols, nsets, nsteps, step,
                       weight, out);
}

__global__ void k_bump(int32_t* step) {
    if (threadIdx.x == 0) *step += 1;
}
__global__ void k_set(int32_t* p, int32_t v) {
    if (threadIdx.x == 0) *p = v;
}
void launch_bump(int32_t* step, hipStream_t s) { hipLaunchKernelGGL(k_bump, dim3(1), dim3(64), 0, s, step); }
void launch_set_scalar(int32_t* p, int32_t v, hipStream_t s) {
    hipLaunchKernelGGL(k_set, dim3(1), dim3(64), 0, s, p, v);
}

// Adjoint RK4 stage combination for active sets:
//   lam_new (=|+=) u ;  mu = alpha * lam + beta * u
__global__ void k_adj_combine(int64_t n, int32_t nsets, const int32_t* nsteps, const int32_t* step,
                              const double* lam, const double* u, double* lam_new, double* mu,
                              double alpha, double beta, int first) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int s = (int)(q % nsets);
    if (nsteps[s] <= *step) return;
    const double uq = u ? u[q] : 0.0;
    if (first) lam_new[q] = lam[q] + uq;
    else lam_new[q] += uq;
    if (mu) mu[q] = alpha * lam[q] + beta * uq;
}

void launch_adj_combine(int64_t rows, int32_t ncols, int32_t nsets, const int32_t* nsteps,
                        const int32_t* step, const double* lam, const double* u, double* lam_new,
                        double* mu, double alpha, double beta, int first, hipStream_t s) {
    const int64_t n = rows * ncols;
    hipLaunchKernelGGL(k_adj_combine, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, nsets, nsteps,
                       step, lam, u, lam_new, mu, alpha, beta, first);
}

__global__ void k_copy_active(int64_t n, int32_t nsets, const int32_t* nsteps, const int32_t* step,
                              const double* src, double* dst) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    if (nsteps[q % nsets] <= *step) return;
    dst[q] = src[q];
}

void launch_copy_active(int64_t rows, int32_t ncols, int32_t nsets, const int32_t* nsteps,
                        const int32_t* step, const double* src, double* dst, hipStream_t s) {
    const int64_t n = rows * ncols;
    hipLaunchKernelGGL(k_copy_active, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, nsets, nsteps,
                       step, src, dst);
}

// set permutation of a [rows][nops][nsets] state (one thread per element)
__global__ void k_permute_sets(const double* __restrict__ src, double* __restrict__ dst, int64_t n,
                               int32_t nsets, const int32_t* __restrict__ perm, int inverse) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const int64_t base = q - q % nsets;
    const int s = (int)(q % nsets);
    if (inverse) dst[base + perm[s]] = src[q];
    else dst[q] = src[base + perm[s]];
}
void launch_permute_sets(const double* src, double* dst, int64_t rows, int32_t nops, int32_t nsets,
                         const int32_t* perm, bool inverse, hipStream_t s) {
    const int64_t n = rows * nops * nsets;
    if (n == 0) return;
    hipLaunchKernelGGL(k_permute_sets, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, dst, n, nsets,
                       perm, inverse ? 1 : 0);
}

// set columns between layouts of ss and sd sets (one thread per moved element)
__global__ void k_move_sets(const double* __restrict__ src, int32_t ss, double* __restrict__ dst, int32_t sd,
                            int64_t n, int32_t q0, int32_t w, const int32_t* __restrict__ perm, int scatter) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t ro = i / w;  // row * nops + op
    const int32_t q = q0 + (int32_t)(i % w);
    const int32_t mq = perm ? perm[q] : q;
    if (scatter) dst[ro * sd + mq] = src[ro * ss + q];
    else dst[ro * sd + q] = src[ro * ss + mq];
}
void launch_move_sets(const double* src, int32_t ss, double* dst, int32_t sd, int64_t rows, int32_t nops,
                      int32_t q0, int32_t q1, const int32_t* perm, bool scatter, hipStream_t s) {
    const int64_t w = (int64_t)q1 - q0, n = rows * nops * w;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_move_sets, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src, ss, dst, sd, n, q0,
                       (int32_t)w, perm, scatter ? 1 : 0);
}

__global__ void k_finite(const double* z, int64_t n, int32_t* flag) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n && !__builtin_isfinite(z[q])) *flag = 1;
}
void launch_finite_check(const double* z, int64_t n, int32_t* flag, hipStream_t s) {
    hipLaunchKernelGGL(k_finite, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, z, n, flag);
}

}  // namespace cut
