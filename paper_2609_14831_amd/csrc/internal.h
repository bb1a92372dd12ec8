// Internal declarations of libcutgraph (host + device).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
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

// ---------------------------------------------------------------- bundle ----
// File layout (little-endian): BundleHeader at 0, then 64-byte aligned
// sections listed by the section table that follows the header.
constexpr char kMagic[8] = {'C', 'U', 'T', 'G', 'R', 'P', 'H', '1'};
constexpr uint32_t kVersion = 1;

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
    SEC_COUNT = 11
};

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
    int32_t factor_bytes;    // 1: int8 integer factors
    int32_t gen_sign;        // +1 / -1
    uint32_t n_sections;
    uint32_t reserved;
    uint64_t section_table_offset;
    uint64_t file_bytes;
    uint64_t records_checksum;
    char identifier[96];
    uint64_t header_checksum;  // of the header with this field zero
    uint8_t pad[256 - 8 - 4 - 4 - 4 - 4 - 8 * 4 - 4 - 4 - 4 - 4 - 8 * 3 - 96 - 8];
};
static_assert(sizeof(BundleHeader) == 256, "header must be 256 bytes");

uint64_t checksum64(const void* data, uint64_t bytes);

// host-side view of a bundle (owned vectors or a mapped file)
struct HostGraph {
    BundleHeader hdr{};
    const uint64_t* labels = nullptr;
    const uint8_t* diag = nullptr;
    const int32_t* pairs = nullptr;
    const int64_t* off[2] = {nullptr, nullptr};
    const int32_t* ri[2] = {nullptr, nullptr};
    const int32_t* rj[2] = {nullptr, nullptr};
    const int8_t* rc[2] = {nullptr, nullptr};
    void* map = nullptr;
    size_t map_bytes = 0;
    ~HostGraph();
};

// Maps and validates a bundle file; throws Fail.
void read_bundle(const char* path, bool verify_checksums, HostGraph& out);

// ------------------------------------------------------------- device side --
// One record stream grouped by output segment.  Each record is a uint2:
// .x = (factor code << 24) | a,  .y = b, where a indexes the "left" operand
// (broadcast over ops) and b the "right" operand of that traversal.
struct Task {          // one workgroup of 4 wavefronts
    int32_t seg;       // first segment
    int32_t nseg;      // >0: that many short segments, one per wavefront;
                       // <0: one long segment split over the 4 wavefronts
};

struct DevCSR {
    int64_t nseg = 0, nrec = 0, max_len = 0;
    int64_t* off = nullptr;     // device [nseg+1]
    uint2* rec = nullptr;       // device [nrec]
    Task* tasks = nullptr;      // device [ntasks] (8*per_xcd when XCD-remapped)
    int64_t ntasks = 0;
    int64_t per_xcd = 0;        // >0: block b runs task (b%8)*per_xcd + b/8
    std::vector<int64_t> off_h; // host copy of the offsets (tiling plan input)
    void release();
};

struct Workspace {
    void* ptr = nullptr;
    size_t bytes = 0;
    void* get(size_t need);     // grows (synchronising) when too small
    void release();
};

struct StepGraphCache;

struct Graph {
    int device = 0;
    BundleHeader hdr{};
    int64_t N = 0;
    double gen_sign = 1.0;
    int nfactors = 0;
    double* ftab = nullptr;          // device [256]
    // record streams: [set][orientation] set 0 = E_L, 1 = E_eta;
    // orientation 0 = by target k (a=i, b=j), 1 = by right input j (a=i, b=k),
    // 2 = by left input i (a=k, b=j)
    DevCSR csr[2][3];
    bool have_adjoint = false;
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
    int xcd_remap = 0;
    Workspace ws;                    // flow state and stage storage
    Workspace ws_small;              // scratch of single generator-VJP calls
    StepGraphCache* graphs = nullptr;
    cut_flow_timing timing{};        // last timed flow
    ~Graph();
};

// tiling plan (host) -> device task list
void build_tasks(Graph& g, DevCSR& c);

// --------------------------------------------------------------- kernels ----
enum Mode { MODE_BCAST = 0, MODE_REDOPS = 1 };
enum Epi { EPI_Y = 0, EPI_ETA = 1, EPI_RK = 2 };

struct PassArgs {
    const DevCSR* csr;
    const double* ftab;
    const void* A;
    int64_t lda;
    const void* B;
    int64_t ldb;
    int32_t nsets, nops;
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

void launch_g2(const Graph& g, double delta, int32_t nsets, const double* h, int64_t ldh,
               void* eta, int64_t lde, bool eta_f32, const int32_t* nsteps, const int32_t* step,
               hipStream_t s);
void launch_g2_vjp(const Graph& g, double delta, int32_t nsets, const double* h, int64_t ldh,
                   const double* gbar, int64_t ldg, double* g_h, int64_t ldgh, double* tmp,
                   hipStream_t s);

// elementwise helpers
void launch_prep_state(const double* z, int64_t rows, int32_t nops, int32_t nsets, void* xsh,
                       bool f32, double* hst, hipStream_t s);
void launch_bump(int32_t* step, hipStream_t s);
void launch_set_scalar(int32_t* p, int32_t v, hipStream_t s);
void launch_adj_combine(int64_t rows, int32_t ncols, int32_t nsets, const int32_t* nsteps,
                        const int32_t* step, const double* lam, const double* u, double* lam_new,
                        double* mu, double alpha, double beta, int first, hipStream_t s);
void launch_copy_active(int64_t rows, int32_t ncols, int32_t nsets, const int32_t* nsteps,
                        const int32_t* step, const double* src, double* dst, hipStream_t s);
void launch_finite_check(const double* z, int64_t n, int32_t* flag, hipStream_t s);

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
struct DeviceGuard {
    int prev = -1;
    explicit DeviceGuard(int dev);
    ~DeviceGuard();
};

}  // namespace cut
