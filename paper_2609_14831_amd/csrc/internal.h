// Internal declarations of libcutgraph (host + device).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <new>
#include <string>
#include <vector>

#include "../../include/cutgraph.h"

namespace cut {

// ---------------------------------------------------------------- errors ----
void set_error(const char* fmt, ...);
struct Fail {
    cut_status st;
};
#define CUT_FAIL(status, ...)          \
    do {                               \
        ::cut::set_error(__VA_ARGS__); \
        throw ::cut::Fail{status};     \
    } while (0)
#define HIP_CHECK(expr)                                                                  \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            CUT_FAIL(CUT_E_DEVICE, "%s: %s (%s:%d)", #expr, hipGetErrorString(e_), __FILE__, \
                     __LINE__);                                                          \
    } while (0)
// body of an extern "C" entry point: no exception crosses the ABI
#define ABI_BEGIN try {
#define ABI_END                                   \
    return CUT_OK;                                \
    }                                             \
    catch (const ::cut::Fail& f) {                \
        return f.st;                              \
    }                                             \
    catch (const std::bad_alloc&) {               \
        ::cut::set_error("out of host memory");   \
        return CUT_E_NOMEM;                       \
    }

// ---------------------------------------------------------------- bundle ----
// File layout (little-endian): BundleHeader at 0, then 64-byte aligned
// sections listed by the section table that follows the header.
constexpr char kMagic[8] = {'C', 'U', 'T', 'G', 'R', 'P', 'H', '1'};
constexpr uint32_t kVersion = 2;

enum SectionId : uint32_t {
    SEC_LABELS = 1,    // uint64[N] registry labels (Majorana bitmask; E_pq p<<32|q)
    SEC_DIAG = 2,      // uint8[N] block-diagonal mask D
    SEC_PAIRS = 3,     // int32[n_pairs] diagonal quadratic coordinates
    SEC_FLOW_OFF = 4,  // int64[N+1]
    SEC_FLOW_I = 5,    // int32[E]
    SEC_FLOW_J = 6,    // int32[E]
    SEC_FLOW_C = 7,    // int8[E]
    SEC_GEN_OFF = 8,   // int64[N+1]
    SEC_GEN_I = 9,     // int32[Eg]
    SEC_GEN_J = 10,    // int32[Eg]
    SEC_GEN_C = 11,    // int8[Eg]
    SEC_COUNT = 11,    // sections of every bundle
    // optional outside-space set E_C (Majorana graphs built with CUT_BUILD_OUTSIDE)
    SEC_OUT_LABELS = 12,  // uint64[Nc] outside registry labels (6-subset bitmasks)
    SEC_OUT_OFF = 13,     // int64[Nc+1]
    SEC_OUT_I = 14,       // int32[Ec]
    SEC_OUT_J = 15,       // int32[Ec]
    SEC_OUT_C = 16,       // int8[Ec]
    SEC_COUNT_OUT = 16,   // sections of a bundle with E_C
    // generator registry labels, present when the generator has a registry of
    // its own (Pauli-boson graphs); placed after the base sections
    SEC_GEN_LABELS = 17   // uint64[NG]
};
constexpr int kMaxSections = 17;

struct SectionEntry {
    uint32_t id;
    uint32_t elem_bytes;
    uint64_t offset;
    uint64_t count;
    uint64_t checksum;
};

struct BundleHeader {
    char magic[8];
    uint32_t version;
    uint32_t header_bytes;
    int32_t algebra;
    int32_t size;
    int64_t n_ops;
    int64_t n_records;
    int64_t n_gen_records;
    int64_t n_pairs;
    int32_t factor_bytes;    // 1: int8 factors; 4: int16 (re, im); 16: FP64 (re, im)
    int32_t gen_sign;        // +1 / -1
    uint32_t n_sections;
    uint32_t reserved;
    uint64_t section_table_offset;
    uint64_t file_bytes;
    uint64_t records_checksum;
    char identifier[96];
    uint64_t header_checksum;  // of the header and section table with this field zero
    int64_t n_out_ops;         // outside registry size (0: no E_C)
    int64_t n_out_records;     // |E_C|
    int64_t n_gen_ops;         // generator registry size (0: the operator registry)
    uint8_t pad[256 - 8 - 4 - 4 - 4 - 4 - 8 * 4 - 4 - 4 - 4 - 4 - 8 * 3 - 96 - 8 - 8 * 3];
};
static_assert(sizeof(BundleHeader) == 256, "header must be 256 bytes");

uint64_t checksum64(const void* data, uint64_t bytes);

// host-side view of a bundle (owned vectors or a mapped file)
struct HostGraph {
    BundleHeader hdr{};
    const uint64_t* labels = nullptr;
    const uint8_t* diag = nullptr;
    const int32_t* pairs = nullptr;
    // record sets: 0 = E_L, 1 = E_eta, 2 = E_C (absent: null, size 0).  Factors
    // are int8 (factor_bytes 1) or, in Pauli-boson graphs, (re, im) pairs of
    // int16 (factor_bytes 4) or of FP64 (factor_bytes 16, registries whose
    // factors leave int16); rc points at the raw bytes.
    const int64_t* off[3] = {nullptr, nullptr, nullptr};
    const int32_t* ri[3] = {nullptr, nullptr, nullptr};
    const int32_t* rj[3] = {nullptr, nullptr, nullptr};
    const int8_t* rc[3] = {nullptr, nullptr, nullptr};
    const uint64_t* out_labels = nullptr;
    const uint64_t* gen_labels = nullptr;
    int64_t n_gen = 0;               // generator rows (the operator registry size when shared)
    void* map = nullptr;
    size_t map_bytes = 0;
    ~HostGraph();
};

// Maps and validates a bundle file; throws Fail.
void read_bundle(const char* path, bool verify_checksums, HostGraph& out);

// ------------------------------------------------------------- device side --
// One record stream grouped by output segment.  Each record is a uint2:
// .x = (f_hi << 24) | a,  .y = (f_lo << 24) | b, where a indexes the "left"
// operand (broadcast over ops) and b the "right" operand of that traversal, and
// (f_hi, f_lo) are the two bytes of the factor's bf16 bit pattern.
struct Task {          // one workgroup of 4 wavefronts
    int32_t seg;       // first segment
    int32_t nseg;      // >0: that many short segments, one per wavefront;
                       // <0: one long segment split over the 4 wavefronts
};

// A chunk of a segment: records [e0, e1) of segment `seg`, summed by one
// wavefront into partial row `slot` (seg < 0: padding, no work).
struct ChunkTask {
    int32_t seg;
    int32_t slot;
    int32_t e0;
    int32_t e1;
};

// Chunked form of a forward pass: chunk tasks (a range of one segment's
// records, summed into a partial row), packed tasks over the remaining short
// segments, and per chunked segment the partial-row slots [cstart[l],
// cstart[l+1]) added in order into row crow[l].
struct ChunkPlan {
    ChunkTask* chunks = nullptr;
    int64_t nchunks = 0;        // including the padding of the XCD split
    Task* short_tasks = nullptr;
    int64_t nshort = 0, short_per_xcd = 0;
    int64_t* cstart = nullptr;  // device [nlong+1]
    int32_t* crow = nullptr;    // device [nlong]
    int64_t nlong = 0;
    int64_t nslots = 0;         // partial rows
    void release();
};

struct DevCSR {
    int64_t nseg = 0, nrec = 0, max_len = 0;
    int64_t* off = nullptr;     // device [nseg+1]
    uint2* rec = nullptr;       // device [nrec]
    Task* tasks = nullptr;      // device [ntasks] (8*per_xcd when XCD-remapped)
    int64_t ntasks = 0;
    int64_t per_xcd = 0;        // >0: block b runs task (b%8)*per_xcd + b/8
    // chunked form (forward passes over E_L): long segments as chunk tasks
    // placed by relative position in their segment, so concurrently running
    // chunks sweep the same operand region
    ChunkPlan cp;
    std::vector<int64_t> off_h; // host copy of the offsets (tiling plan input)
    // Pauli-boson E_L / E_C: the same records in complex form, grouped by
    // complex target (FP64 forward passes run over these; see k_cpass)
    const DevCSR* cx = nullptr;
    int64_t na = 0, nb = 0;     // complex twins: rows of the left / right input space
    // rows of the largest array a pass over these records reads (targets, left
    // or right inputs; 0: the segment count), for the 32-bit offset check
    int64_t rows = 0;
    void release();
};

// Shared-triple tiles (Majorana registries).  Every record of a quartic target
// K pairs a quadratic string with a quartic K' sharing three modes tau = K & K'.
// Tile tau owns the M = m-3 quartic rows tau+w (w not in tau): they are both the
// tile's targets and the quartic operands of its records, so one workgroup
// stages them in LDS once.  Record of member t: .x = quadratic row, .y =
// (top half of the FP32 factor << 16) | (local operand q << 1) | orient (0:
// generator from the quadratic row, operand from LDS; 1: generator from LDS,
// operand from the quadratic row); the orient-0 records form the first half.
// Target tau+w receives its tile-tau sum in partial slot `slot` (the position
// of w in K); the 4 slots are added in fixed order by the combine.
struct TilePlan {
    int64_t ntiles = 0;
    int32_t M = 0;             // members per tile
    int32_t RT = 0;            // records per member
    int64_t nres = 0;          // segments [0, nres) stay with the segment kernel
    int32_t* rows = nullptr;   // device [ntiles * M]
    uint8_t* slot = nullptr;   // device [ntiles * M]
    uint2* rec = nullptr;      // device [ntiles * M * RT]
    Task* res_tasks = nullptr; // segment tasks over [0, nres)
    int64_t nres_tasks = 0;
    int64_t res_per_xcd = 0;
    bool ok = false;
    void release();
};

// Blocks of quadratic targets (Majorana registries).  Beyond its leading
// quadratic x quadratic records, quadratic target {u, v} (u < v) holds, for
// every triple T of modes outside {u, v} in lexicographic order, the record
// pair (T+u, T+v), (T+v, T+u) -- checked record by record at load.  Modes are
// grouped by 8; one workgroup owns the targets {u, v} with u in group g1 and v
// in group g2 (g1 <= g2, at most 64) and a range of triples: per triple it
// stages the <= 16 rows T+w of its modes in LDS, so each row feeds up to 16
// records from LDS instead of 16 gathers, and the targets' sums stay in
// registers across the range; each (target, range) sum is one partial row.
// The records' factors are re-encoded at load as sign bits per (group pair,
// wavefront, triple) with one common magnitude (checked against every record).
struct QuadBlockPlan {
    bool ok = false;
    int32_t m = 0, ng = 0, nbp = 0, nr = 0;  // modes, mode groups, group pairs, triple ranges
    int64_t ntrip = 0;
    int32_t* row4 = nullptr;     // device [ntrip * m]: row of T+w, -1 when w is in T
    uint64_t* tmask = nullptr;   // device [ntrip]: mode mask of triple T
    int2* bpair = nullptr;       // device [nbp]: first modes of group 1 and group 2
    uint32_t* sgn = nullptr;     // device [nbp * 8 * ntrip]: sign bits of the records of
                                 // wavefront w's targets at triple T (2 per target: bit 2j
                                 // for (T+u, T+v), bit 2j+1 for (T+v, T+u)), 1 = negative
    float fmag = 0.f;            // common magnitude of those factors
    std::vector<int32_t> qrow;   // host: quadratic target rows, by pair (u, v) as u * m + v
    std::vector<int32_t> lead;   // host [N]: leading records of quadratic target rows
    // per tiling (rebuilt with the task lists)
    int32_t* tslot = nullptr;    // device [nbp * 64]: first block partial slot, -1 no target
    ChunkPlan cp;                // leading records of the quadratic targets + the rest
    ChunkPlan cp_lead;           // leading records only (quartic targets in tiles)
    bool active = false;         // plan built for the current tiling
    void release_tiling();
    void release();
};

// Device work area of a graph handle.  It is sized only by reservation calls
// (cut_graph_reserve, and the tiling calls that re-size it for the shapes
// reserved so far); the computing entry points take their share with need(),
// which never allocates or synchronises and fails with CUT_E_INVAL when the
// reservation is too small.
struct Workspace {
    void* ptr = nullptr;
    size_t bytes = 0;
    void* need(size_t n, const char* what) const;
    void reserve(size_t n);     // grows: synchronises the device, frees, allocates
    void release();
};

struct StepGraphCache;

struct Graph {
    int device = 0;
    BundleHeader hdr{};
    int64_t N = 0;                   // operator rows (Pauli-boson: 2 x labels, real-split)
    int64_t NG = 0;                  // generator rows (= N unless the generator has its own registry)
    double gen_sign = 1.0;
    int nfactors = 0;
    double* ftab = nullptr;          // device [256]: factor dictionary of the stencil tables
    // record streams: [set][orientation] set 0 = E_L, 1 = E_eta, 2 = E_C
    // (orientation 0 only, segments = outside registry rows);
    // orientation 0 = by target k (a=i, b=j), 1 = by right input j (a=i, b=k),
    // 2 = by left input i (a=k, b=j)
    DevCSR csr[3][3];
    DevCSR cxs[3];                   // complex twins of the record sets (Pauli-boson only)
    bool have_adjoint = false;
    bool have_outside = false;
    int64_t n_out = 0;               // outside rows (Pauli-boson: 2 x labels)
    std::vector<uint64_t> gen_labels_h, out_labels_h;   // host copies (generator registry only when own)
    // block mask and pairs
    uint8_t* diag = nullptr;         // device [N]
    int32_t* pairs = nullptr;        // device [npairs]
    int64_t npairs = 0;
    // G2 stencil: per target up to 4 entries (partner, pair, factor)
    int4* stencil = nullptr;         // device [N*4]: x partner (-1 = none), y pair a, z factor code
    int64_t* st_t_off = nullptr;     // transposed stencil CSR [N+1]
    int4* st_t = nullptr;            // entries: x = S, y = pair a, z = factor code (of S's entry)
    int64_t* st_p_off = nullptr;     // per-pair list CSR [npairs+1]
    int4* st_p = nullptr;            // entries: x = S, y = partner, z = factor code
    bool have_stencil = false;
    int64_t long_records = 1024;
    int64_t chunk_records = 512;     // records per chunk of a long target
    int xcd_remap = 0;
    int triple_chunks = 0;           // cut quartic Majorana targets by shared triple
    // Majorana quartic targets whose records come in 4 equal shared-triple
    // groups, in ascending triple rank (checked at load)
    bool triple_groups = false;
    std::vector<uint64_t> labels_h;  // registry labels (host copy)
    TilePlan tiles;
    int use_tiles = 0;
    QuadBlockPlan qb;
    int use_quadblocks = 0;
    uint64_t tiling_gen = 0;         // bumped whenever task lists are rebuilt
    int use_chunks = 1;
    int bchunk = 0;                  // B-chunk field of the tiling flags: lane groups of <= 64 >> bchunk sets
    int64_t max_lds = 65536;         // LDS bytes one workgroup may allocate
    Workspace ws;                    // flow state and stage storage
    Workspace ws_small;              // scratch of single generator-VJP calls
    Workspace ws_part;               // tile partial slots of single forward passes
    Workspace ws_deriv;              // generator, tangent and float shadows of derivative calls
    // shapes reserved so far: (nsets, nops, ckpt_every, CUT_RESERVE_* flags)
    std::vector<std::vector<int64_t>> reserved;
    StepGraphCache* graphs = nullptr;
    // host copies the last flow uploaded (kept alive past the asynchronous copies)
    std::vector<int32_t> flow_perm_h, flow_nsteps_h;
    cut_flow_timing timing{};        // last timed flow
    std::vector<std::pair<std::vector<int64_t>, cut_tuning>> tune_cache;
    ~Graph();
};

// work-area sizes (bytes) of the computing entry points for one shape and
// precision; reserve_shape() grows every work area to the largest over the
// precisions, rereserve() repeats that for every shape reserved so far (after
// the tiling, and with it the partial-row count, changed)
size_t flow_ws_bytes(const Graph& g, int64_t nsets, int64_t nops, int prec, size_t extra);
size_t flow_outside_extra(const Graph& g, int64_t nsets, int64_t nops);
size_t flow_adjoint_extra(const Graph& g, int64_t nsets, int64_t nops, int64_t ckpt_every);
size_t jvp_ws_bytes(const Graph& g, int64_t nsets, int64_t nops, int prec);
size_t vjp_ws_bytes(const Graph& g, int64_t nsets, int64_t nops, int prec);
void reserve_shape(Graph& g, int64_t nsets, int64_t nops, int64_t ckpt_every, uint32_t what);
void rereserve(Graph& g);

// tiling plan (host) -> device task list
void build_tasks(Graph& g, DevCSR& c);
// sets the tiling parameters and rebuilds the task lists of every loaded copy
void apply_tiling(Graph& g, int64_t long_records, int64_t chunk_records, uint32_t flags);
uint32_t tiling_flags(const Graph& g);

// --------------------------------------------------------------- kernels ----
enum Mode { MODE_BCAST = 0, MODE_REDOPS = 1 };
enum Epi { EPI_Y = 0, EPI_ETA = 1, EPI_RK = 2 };

struct PassArgs {
    const DevCSR* csr;
    const Task* tasks = nullptr;    // overrides csr's task list when set
    int64_t ntasks = 0;
    int64_t per_xcd = 0;
    const void* A;
    int64_t lda;
    const void* B;
    int64_t ldb;
    int32_t nsets, nops;
    int32_t s0 = 0, s1 = 0;         // sets [s0, s1) covered (s1 = 0: all); see forward_set_ranges
    int32_t gmax = 64;              // widest lane group of the segment kernel (the tiling's B-chunk)
    // 1: a full-width forward pass takes the segment kernel over the chunk plan
    // (the route of a launch over a proper set range) instead of the tiling's
    // block and tile kernels, whose lanes are sets (a ragged flow's compacted
    // narrow phase)
    int32_t narrow = 0;
    // lane groups of the segment kernel span at least this many sets (a
    // compacted flow keeps the widths, hence the sums, of its full layout)
    int32_t gfloor = 1;
    int32_t precision;              // cut_precision
    const int32_t* nsteps;          // device [nsets] or null (all active)
    const int32_t* step;            // device scalar or null
    // EPI_Y / EPI_ETA
    void* y;
    int64_t ldy;
    int32_t accumulate;
    double scale;
    // EPI_RK
    int32_t stage;
    double ds;
    double* z;
    double* acc;
    void* xout;                     // next-stage operand shadow (ld = ldb)
    double* hst;                    // FP64 Hamiltonian column of the next stage
    int64_t ldh;
};

void launch_pass(int mode, int epi, const PassArgs& a, hipStream_t s);

// Forward pass of record set 0 over every target: the shared-triple tile path
// when available for this shape (residual segment kernel + tile kernel +
// fixed-order combine with the epilogue), otherwise the segment kernel.
// `partials` must hold tile_partial_bytes() bytes when the tile path is taken.
bool tiles_usable(const Graph& g, int32_t nsets, int32_t nops, int32_t precision);
// bytes of partial rows the chunked forward pass needs (0: not chunked)
size_t chunk_partial_bytes(const Graph& g, int32_t nsets, int32_t nops);
// partial work area a forward pass of record set 0 needs (tiles or chunks)
size_t forward_partial_bytes(const Graph& g, int32_t nsets, int32_t nops, int32_t precision);
size_t tile_partial_bytes(const Graph& g, int32_t nsets, int32_t nops);
bool quadblocks_usable(const Graph& g, int32_t nsets, int32_t nops, int32_t precision);
void launch_forward(const Graph& g, int epi, const PassArgs& a, double* partials, hipStream_t s);
bool forward_set_ranges(const Graph& g, const PassArgs& a);
// rows x (nops x nsets) state: dst[r][op][s] = src[r][op][perm[s]] (inverse:
// dst[r][op][perm[s]] = src[r][op][s])
void launch_permute_sets(const double* src, double* dst, int64_t rows, int32_t nops, int32_t nsets,
                         const int32_t* perm, bool inverse, hipStream_t s);
// set columns [q0, q1) between a rows x (nops x ss) state and a rows x
// (nops x sd) one, map(q) = perm[q] (q without perm): gather
// dst[r][op][q] = src[r][op][map(q)], scatter dst[r][op][map(q)] = src[r][op][q]
void launch_move_sets(const double* src, int32_t ss, double* dst, int32_t sd, int64_t rows, int32_t nops,
                      int32_t q0, int32_t q1, const int32_t* perm, bool scatter, hipStream_t s);

void launch_g2(const Graph& g, double delta, int32_t nsets, const double* h, int64_t ldh,
               void* eta, int64_t lde, bool eta_f32, const int32_t* nsteps, const int32_t* step,
               hipStream_t s);
void launch_g2_vjp(const Graph& g, double delta, int32_t nsets, const double* h, int64_t ldh,
                   const double* gbar, int64_t ldg, double* g_h, int64_t ldgh, double* tmp,
                   hipStream_t s);
void launch_g2_jvp(const Graph& g, double delta, int32_t nsets, const double* h, int64_t ldh,
                   const double* dh, int64_t lddh, double* deta, int64_t ldde, hipStream_t s);

void launch_g1(const Graph& g, double delta, int32_t nsets, const double* h, int64_t ldh, void* eta,
               int64_t lde, bool eta_f32, const int32_t* nsteps, const int32_t* step, hipStream_t s);
void launch_g1_jvp(const Graph& g, double delta, int32_t nsets, const double* h, int64_t ldh,
                   const double* dh, int64_t lddh, double* deta, int64_t ldde, hipStream_t s);
void launch_g1_vjp(const Graph& g, double delta, int32_t nsets, const double* h, int64_t ldh,
                   const double* gbar, int64_t ldg, double* g_h, int64_t ldgh, double* tmp, hipStream_t s);
// generators evaluated from the pair-flip stencil (G1, G2): they need scratch
// of 2 N nsets doubles in their VJP
inline bool stencil_generator(int kind) { return kind == CUT_GEN_G1 || kind == CUT_GEN_G2; }

// elementwise helpers
void launch_prep_state(const double* z, int64_t rows, int32_t nops, int32_t nsets, void* xsh,
                       bool f32, double* hst, hipStream_t s);
void launch_round_f32(const double* src, int64_t lds, int64_t rows, int64_t cols, float* dst, int64_t ldd,
                      hipStream_t s);
void launch_zero2d(double* dst, int64_t ld, int64_t rows, int64_t cols, hipStream_t s);
// out[c] += weight * sum_r y[r][c]^2 for columns of active sets (fixed order;
// part holds nparts * cols doubles)
constexpr int32_t kColsqParts = 1024;
void launch_colsq_accumulate(const double* y, int64_t rows, int64_t cols, int32_t nsets, double* part,
                             int32_t nparts, const int32_t* nsteps, const int32_t* step, double weight,
                             double* out, hipStream_t s);
void launch_bump(int32_t* step, hipStream_t s);
void launch_set_scalar(int32_t* p, int32_t v, hipStream_t s);
void launch_adj_combine(int64_t rows, int32_t ncols, int32_t nsets, const int32_t* nsteps,
                        const int32_t* step, const double* lam, const double* u, double* lam_new,
                        double* mu, double alpha, double beta, int first, hipStream_t s);
void launch_copy_active(int64_t rows, int32_t ncols, int32_t nsets, const int32_t* nsteps,
                        const int32_t* step, const double* src, double* dst, hipStream_t s);
void launch_finite_check(const double* z, int64_t n, int32_t* flag, hipStream_t s);

// validated pass arguments of a forward action (cut_graph_apply and its
// allocation-free variant); *part_bytes = partial-row bytes it needs
PassArgs apply_args(Graph& g, int32_t which, int32_t precision, int64_t nsets, int64_t nops, const void* eta,
                    int64_t lde, const void* x, int64_t ldx, double* y, int64_t ldy, uint32_t flags,
                    size_t* part_bytes);

// shared by the ABI entry points (capi.cpp) and the flow driver (flow.cpp)
Graph& checked(cut_graph_t h);
void check_prec(int p);
void check_shape(int64_t nsets, int64_t nops);
void check_generator(const Graph& g, int kind);
void eval_generator(Graph& g, int kind, double delta, int32_t nsets, const double* h, int64_t ldh, void* eta,
                    int64_t lde, bool eta_f32, const int32_t* nsteps, const int32_t* step, hipStream_t s);
void eval_generator_vjp(Graph& g, int kind, double delta, int32_t nsets, const double* h, int64_t ldh,
                        const double* gbar, int64_t ldg, double* g_h, int64_t ldgh, double* tmp,
                        hipStream_t s);
void eval_generator_jvp(Graph& g, int kind, double delta, int32_t nsets, const double* h, int64_t ldh,
                        const double* dh, int64_t lddh, double* deta, int64_t ldde, hipStream_t s);
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev);
    ~DeviceGuard();
};

}  // namespace cut
