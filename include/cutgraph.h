/* cutgraph.h -- C ABI of the MI355X compiled-CUT-graph library (libcutgraph.so).
 *
 * Method: Peng & Govind, "Compile-once operation graphs for reusable continuous
 * unitary transformations".  A fixed operator registry and transformation rule
 * are compiled once into a graph of contribution records (target k, left input
 * i, right input j, factor c), grouped by target (Sec. 2.2, Eq. graph-actions).
 * Evaluating the graph on run-time coefficient vectors gives the projected flow
 * right-hand side dh_k/ds = sum_e c_e eta_{i_e} h_{j_e} for [eta, H] and [eta, X]
 * (Sec. 2.1, Eq. coflow); the same records, traversed toward their inputs, give
 * the adjoint action (Sec. 2.4).
 *
 * Conventions for every entry point:
 *  - Status codes are returned; nothing throws across the ABI.  After a non-OK
 *    status, cut_last_error() returns a thread-local message.
 *  - Argument and shape validation is synchronous and happens before any launch
 *    (CUT_E_INVAL).  Kernels run asynchronously on `stream` (a hipStream_t;
 *    NULL = the null stream).  A device fault surfaces as CUT_E_DEVICE from a
 *    later call that synchronises.
 *  - All coefficient pointers are device memory owned by the caller.  Row r of
 *    an operand starts at base + r*ld (ld counted in elements).  Leading
 *    dimensions are below 2^31 elements (the kernels form row addresses from
 *    32-bit strides); larger ones fail with CUT_E_INVAL before any launch.
 *  - Coefficient layout: a state row holds nops*nsets columns, column
 *    op*nsets + s belongs to operand op (0 = the Hamiltonian) of coefficient set
 *    s.  A generator row holds nsets columns.  Every operand column of set s is
 *    paired with generator column s.
 *  - A graph handle owns all device copies of the graph and its work areas.
 *    Work areas are sized only by cut_graph_reserve (and re-sized by the
 *    tiling calls for the shapes reserved so far).  The computing entry points
 *    -- cut_graph_apply, cut_graph_apply_adjoint, cut_generator*,
 *    cut_graph_jvp/vjp, cut_flow_integrate, cut_flow_adjoint -- never allocate
 *    device memory and never synchronise the device; a shape that was not
 *    reserved fails with CUT_E_INVAL before any launch.
 *  - Concurrency: the graph's records and plans are read-only during
 *    computing calls, but the work areas are shared by every call on one
 *    handle.  Calls that use a work area (chunked forward passes, generator
 *    VJP, derivatives, flows) must not overlap in time on one handle: issue
 *    them on one stream, or load the bundle once per stream.  Setup calls
 *    (reserve, set_tiling, autotune, free) must not run concurrently with any
 *    other call on the handle.
 */
#ifndef CUTGRAPH_H
#define CUTGRAPH_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cut_graph_s* cut_graph_t;

typedef enum {
    CUT_OK = 0,
    CUT_E_INVAL = 1,        /* bad argument, shape or leading dimension */
    CUT_E_IO = 2,           /* file cannot be created, read or mapped */
    CUT_E_FORMAT = 3,       /* bundle header/section/bounds validation failed */
    CUT_E_CHECKSUM = 4,     /* bundle section checksum mismatch */
    CUT_E_NOMEM = 5,        /* host or device allocation failed */
    CUT_E_DEVICE = 6,       /* HIP runtime error or device fault */
    CUT_E_NUMERIC = 7,      /* non-finite state detected by a flow */
    CUT_E_UNSUPPORTED = 8   /* valid request outside what this library implements */
} cut_status;

/* Operator algebras the graph compiler knows. */
typedef enum {
    CUT_ALG_EPQ = 1,        /* one-body fermion operators E_pq, size = n orbitals,
                               registry index p*n+q, [E_pq,E_rs] = d_qr E_ps - d_ps E_rq */
    CUT_ALG_MAJORANA = 2,   /* even Majorana strings of degree 2 and 4 over m = size
                               modes, registry = 2-subsets then 4-subsets, each
                               lexicographic; generator basis i*Gamma_S */
    CUT_ALG_PAULI_BOSON = 3 /* Pauli-boson labels B_{tau,c,a} = sigma_tau prod_m
                               (b_m^+)^{c_m} b_m^{a_m} (Eq. monomial) over M boson
                               modes, the complete degree-p registry |c|+|a| <= p
                               (4 C(2M+p, p) labels, Eq. basis-size); size =
                               256 M + p (M in 1..5).  Complex coefficients; the
                               generator [H_d, H_od] has a registry of its own.
                               Factors are Gaussian integers, exact in 128-bit
                               arithmetic during compilation and stored as int16
                               (re, im) pairs, or as the nearest FP64 pairs when
                               one leaves int16 (M = 1 from p = 8; the degree-24
                               one-mode registry reaches ~2e37) */
} cut_algebra;

/* Record sets stored in a graph (Eq. graph-actions). */
typedef enum {
    CUT_GRAPH_FLOW = 0,     /* E_L: the retained action F_k(h, x) */
    CUT_GRAPH_GEN = 1,      /* E_eta: block-generator records (left input diagonal) */
    CUT_GRAPH_OUTSIDE = 2   /* E_C: the optional outside-space action C_q(h, x)
                               (Eq. projected-flow; Eq. graph-actions, third line);
                               targets are the outside registry rows */
} cut_which;

/* Arithmetic of a graph pass. */
typedef enum {
    CUT_F64 = 0,            /* double operands, double products and sums */
    CUT_F32C = 1,           /* float operands and products; compensated sums
                               (error-free product by FMA + two-sum), double result */
    CUT_F32X = 2,           /* float operands; products and sums in double (products
                               of two floats and a small integer factor are exact) */
    CUT_F32 = 3             /* float operands, products and plain float sums
                               (precision-study baseline only) */
} cut_precision;

/* Generators eta(h) (Sec. 2.1, Eq. block-generator). */
typedef enum {
    CUT_GEN_WEGNER_GRAPH = 1, /* eta = [H_d, H_od] as a graph pass over E_eta */
    CUT_GEN_G2 = 2,           /* Majorana: Wegner generator of the quadratic diagonal
                                 part H_0 = sum_a eps_a Gamma_{P_a}, eps_a = h_{P_a},
                                 divided elementwise by Q_S = sum_t (c_t eps_{a_t})^2
                                 + delta^2 (the diagonal of ad_{H_0}^2) */
    CUT_GEN_G1 = 3            /* Majorana: the literal White-type generator from the
                                 diagonal pair energies, eta_S = h_S / D_S with
                                 D_S = 2 sum_{a in F(S)} |eps_a| + delta over the
                                 pairs a that S flips (|S & P_a| = 1); eta = 0 on
                                 block-diagonal strings.  In the string basis it
                                 rotates h_S with its partners S ^ P_a instead of
                                 damping it: kept for the precision study */
} cut_generator_kind;

#define CUT_BUILD_OUTSIDE 1u  /* build flags: also compile the outside-space records */
#define CUT_ACCUMULATE   1u   /* apply flags: y += result instead of y = result */
#define CUT_LOAD_ADJOINT 1u   /* load flags: also build the input-sorted copies */
#define CUT_LOAD_NO_CHECKSUM 2u /* load flags: skip section checksums (bounds are
                                   still validated) */

typedef struct {
    int32_t algebra;        /* cut_algebra */
    int32_t size;           /* n orbitals or m Majorana modes */
    int64_t n_ops;          /* registry size N */
    int64_t n_records;      /* |E_L| */
    int64_t n_gen_records;  /* |E_eta| */
    int64_t n_pairs;        /* diagonal quadratic coordinates (pair energies) */
    int64_t n_out_ops;      /* outside registry size (0 without E_C) */
    int64_t n_out_records;  /* |E_C| */
    int64_t n_gen_ops;      /* generator registry size (0: the operator registry) */
    uint64_t checksum;      /* combined checksum of the record sections */
    int64_t file_bytes;     /* bundle size on disk */
    double build_seconds;   /* compiler wall time (cut_graph_build only) */
    char identifier[96];    /* algebra, registry, ordering and projection rules */
} cut_graph_desc;

/* ---------------------------------------------------------------- compile --
 * cut_graph_build: compile the graph of `algebra` at `size` into a bundle file
 * (Sec. 2.3).  Two deterministic traversals: the first counts the records of
 * every target and fixes the exact array sizes, the file is then sized and
 * mapped, the second traversal writes every record at its final place.  The
 * bundle holds the registry labels, block mask, pair list, rules identifier,
 * factor precision (int8; Pauli-boson: int16 or FP64 pairs, see
 * CUT_ALG_PAULI_BOSON), the target-grouped records of E_L and E_eta and one
 * checksum per section.  Two builds are bitwise identical.
 * With CUT_BUILD_OUTSIDE (Majorana, m <= 32) the bundle also holds the outside
 * registry (every 6-subset of the modes, lexicographic) and the target-grouped
 * records E_C of the degree-6 part of [eta, X] that the projection drops
 * (Eq. projected-flow): two quartics sharing one mode, 20 (m - 6) records per
 * outside target.  They never feed the flow; they give the diagnostic action
 * C_q (Eq. graph-actions, third line).
 * `threads` <= 0 selects the hardware concurrency.  `desc` (nullable) receives
 * the sizes.  Errors: CUT_E_INVAL (unknown algebra or flag, size out of range:
 * E_pq 1..64, Majorana even 4..64; CUT_BUILD_OUTSIDE with E_pq, whose registry
 * is closed), CUT_E_UNSUPPORTED (CUT_BUILD_OUTSIDE above 32 modes; a
 * Pauli-boson registry whose labels do not fit 64 bits or p > 31, or a factor
 * beyond the int128 range), CUT_E_IO, CUT_E_NOMEM. */
cut_status cut_graph_build(int32_t algebra, int32_t size, const char* path, int32_t threads,
                           uint32_t flags, cut_graph_desc* desc);

/* ------------------------------------------------------------------- load --
 * cut_graph_load: map and validate a bundle (magic, version, header checksum,
 * section table, per-section checksums unless CUT_LOAD_NO_CHECKSUM, offsets
 * monotone and complete, every index < N, every factor nonzero), then upload
 * the target-sorted record stream to `hip_device` (Sec. 2.3: validated reload).
 * With CUT_LOAD_ADJOINT the input-sorted copies used by the adjoint are built
 * too.  Outside-space records, when the bundle has them, are uploaded in their
 * target order (forward action only).  A device record carries 8 significant
 * bits of factor; a wider Pauli-boson factor is loaded as several records on
 * the same rows whose factors sum exactly to it (each the remainder truncated
 * to 8 bits: at most 7 for an FP64 factor, all of its sign), so every pass
 * evaluates the stored factor with the error bound of a longer segment.
 * On success *out owns all device memory; release with cut_graph_free.
 * Errors: CUT_E_IO, CUT_E_FORMAT (also a non-finite factor), CUT_E_CHECKSUM,
 * CUT_E_NOMEM, CUT_E_DEVICE, CUT_E_UNSUPPORTED (N >= 2^24, more than 256
 * distinct factors, or a factor piece outside the normal FP32 range). */
cut_status cut_graph_load(const char* path, int32_t hip_device, uint32_t flags, cut_graph_t* out);

cut_status cut_graph_info(cut_graph_t g, cut_graph_desc* desc);

/* cut_graph_labels: copies the labels of a registry into host memory `out` of
 * exactly n entries: which = CUT_GRAPH_FLOW the operator registry (n_ops),
 * CUT_GRAPH_GEN the generator registry (n_gen_ops, or the operator registry
 * when n_gen_ops is 0), CUT_GRAPH_OUTSIDE the outside registry (n_out_ops).
 * Label keys: E_pq p << 32 | q; Majorana the bitmask of the string's modes;
 * Pauli-boson W-bit fields, W the bit length of 3p, from the most significant:
 * total degree, tau (2 bits: 0 = I, 1 = x, 2 = y, 3 = z), then c_1, a_1, ...,
 * c_M, a_M (their numeric order is the registry order).  Pauli-boson
 * coefficient vectors are complex and stored real-split on the device: a
 * registry of n labels has 2n rows, row 2r the real and row 2r + 1 the
 * imaginary part of coefficient r (operands, generator, outputs alike).
 * Errors: CUT_E_INVAL (null argument, unknown or absent registry, n mismatch). */
cut_status cut_graph_labels(cut_graph_t g, int32_t which, uint64_t* out, int64_t n);
void cut_graph_free(cut_graph_t g);

/* ---------------------------------------------------------- work areas --
 * cut_graph_reserve: sizes the handle's work areas for calls with nsets
 * coefficient sets and nops operands per set, in every precision, for the
 * call kinds in `what`:
 *   CUT_RESERVE_APPLY   cut_graph_apply (partial rows of chunked or tiled
 *                       forward passes) and cut_generator_vjp;
 *   CUT_RESERVE_FLOW    cut_flow_integrate (stage operands, RK accumulator,
 *                       generator, step counters; plus the outside-space
 *                       diagnostic buffers when the graph holds E_C);
 *   CUT_RESERVE_DERIV   cut_graph_jvp and cut_graph_vjp;
 *   CUT_RESERVE_ADJOINT cut_flow_adjoint with checkpoints every ckpt_every
 *                       steps (stage storage of one checkpoint block).
 * Work areas only grow; a reservation also covers every smaller nsets / nops.
 * The shape is remembered: cut_graph_set_tiling and cut_graph_autotune
 * re-size the work areas for every shape reserved so far.  Growing
 * synchronises the device and moves the work area (captured flow step graphs
 * are then re-made).  Errors: CUT_E_INVAL (null handle, unknown flag, shape
 * out of range, CUT_RESERVE_ADJOINT with ckpt_every < 1), CUT_E_NOMEM,
 * CUT_E_DEVICE.
 * cut_graph_reserved_bytes: total bytes of the handle's work areas. */
#define CUT_RESERVE_APPLY 1u
#define CUT_RESERVE_FLOW 2u
#define CUT_RESERVE_DERIV 4u
#define CUT_RESERVE_ADJOINT 8u
cut_status cut_graph_reserve(cut_graph_t g, int64_t nsets, int64_t nops, int64_t ckpt_every, uint32_t what);
cut_status cut_graph_reserved_bytes(cut_graph_t g, int64_t* bytes);

/* ------------------------------------------------------------------ apply --
 * cut_graph_apply: forward graph action (Eq. graph-actions; L(h)x of Sec. 2.4)
 *   y[k][op*nsets+s] (=|+=) sum_{e in E(k)} c_e * eta[i_e][s] * x[j_e][op*nsets+s]
 * for 0 <= k < N, 0 <= op < nops, 0 <= s < nsets.  eta and x are double* for
 * CUT_F64 and float* otherwise; y is always double*.  Requires nsets >= 1,
 * 1 <= nops <= 8, lde >= nsets, ldx >= nops*nsets, ldy >= nops*nsets.
 * y must not alias eta or x.  Row counts: x has one row per operator row,
 * eta one per generator row (the same unless the generator has a registry of its
 * own, n_gen_ops > 0), y one per target row: operator rows for CUT_GRAPH_FLOW,
 * generator rows for CUT_GRAPH_GEN (whose inputs are both operator rows), outside
 * rows for CUT_GRAPH_OUTSIDE (CUT_E_INVAL if the bundle has no outside-space
 * records).  Pauli-boson graphs have twice as many rows as labels (real-split,
 * see cut_graph_labels).  Chunked and tiled forward passes over E_L keep
 * partial rows in the work area reserved with CUT_RESERVE_APPLY (CUT_E_INVAL
 * when it was not reserved for this shape). */
cut_status cut_graph_apply(cut_graph_t g, int32_t which, int32_t precision, int64_t nsets,
                           int64_t nops, const void* eta, int64_t lde, const void* x,
                           int64_t ldx, double* y, int64_t ldy, uint32_t flags, void* stream);

/* cut_graph_apply_adjoint: the graph-level adjoint (Sec. 2.4): the same factor,
 * accumulated into the input coordinate (the factors of the real records need
 * no conjugation):
 *   g_x[j][op*nsets+s]  (=|+=) sum_{e: j_e=j} c_e * eta[i_e][s] * w[k_e][op*nsets+s]
 *   g_eta[i][s]         (=|+=) sum_{e: i_e=i} c_e * sum_op w[k_e][op*nsets+s] * x[j_e][op*nsets+s]
 * Either output may be NULL (then its inputs may be NULL too).  Needs a graph
 * loaded with CUT_LOAD_ADJOINT (else CUT_E_INVAL).  Types as cut_graph_apply.
 * which = CUT_GRAPH_OUTSIDE is not supported (CUT_E_INVAL).  On Pauli-boson
 * graphs (real-split rows) this real transpose is the complex adjoint with the
 * conjugation the paper names: g_x[j] = sum conj(c xi_a) w_k and
 * g_eta[a] = sum conj(c x_j) w_k. */
cut_status cut_graph_apply_adjoint(cut_graph_t g, int32_t which, int32_t precision, int64_t nsets,
                                   int64_t nops, const void* eta, int64_t lde, const void* x,
                                   int64_t ldx, const void* w, int64_t ldw, double* g_x,
                                   int64_t ldgx, double* g_eta, int64_t ldge, uint32_t flags,
                                   void* stream);

/* cut_graph_apply_noalloc: cut_graph_apply for callers that cannot allocate
 * device memory or call a reserving entry point first (code under stream
 * capture, tight serving loops, harnesses that forbid allocation).  Same
 * arguments, result and kernels; the partial rows of a chunked or tiled
 * forward pass live in a fixed device array of 64 MiB built into the library
 * (one per GPU, held until the process ends) instead of the handle's work
 * area, so no cut_graph_reserve is needed and nothing is allocated.  Every
 * call on one GPU shares that array (it keeps the last call's partial rows;
 * each call writes every row it reads first), so calls that overlap in time on
 * one GPU race: issue them on one stream.  Errors: as cut_graph_apply, plus
 * CUT_E_INVAL when the shape and tiling need more than 64 MiB of partial rows
 * (fewer columns per call, longer chunks or CUT_TILE_NO_CHUNKS fit). */
cut_status cut_graph_apply_noalloc(cut_graph_t g, int32_t which, int32_t precision, int64_t nsets,
                                   int64_t nops, const void* eta, int64_t lde, const void* x, int64_t ldx,
                                   double* y, int64_t ldy, uint32_t flags, void* stream);

/* -------------------------------------------------------------- generator --
 * cut_generator: eta[r][s] from h[r][s] (both double with leading dimensions;
 * h has the operator rows, eta the generator rows), for CUT_GEN_WEGNER_GRAPH
 * (eta_k = s_g sum_{E_eta(k)} c (Dh)_i ((I-D)h)_j, s_g = +1 for E_pq and
 * Pauli-boson labels, -1 for Majorana strings, whose generator basis is
 * i*Gamma), CUT_GEN_G2 or CUT_GEN_G1 (Majorana only; eta = 0 on diagonal
 * strings).
 * cut_generator_vjp: g_h[r][s] += sum_S gbar[S][s] d eta_S / d h_r. */
cut_status cut_generator(cut_graph_t g, int32_t kind, double delta, int64_t nsets,
                         const double* h, int64_t ldh, double* eta, int64_t lde, void* stream);
cut_status cut_generator_vjp(cut_graph_t g, int32_t kind, double delta, int64_t nsets,
                             const double* h, int64_t ldh, const double* gbar, int64_t ldg,
                             double* g_h, int64_t ldgh, void* stream);

/* ------------------------------------------------------------ derivatives --
 * Derivatives of one projected action F(h, x) = L(eta(h)) x (Sec. 2.4,
 * Eq. directional-derivative): h is the Hamiltonian column that defines the
 * generator ([N][nsets], double), x the operand ([N][nops*nsets], double, in
 * the layout of cut_graph_apply).  x is independent of h here; to differentiate
 * the Hamiltonian's own right-hand side pass h also as operand 0 and dh also as
 * its tangent.  The generator is `kind` with regulariser `delta` as in
 * cut_generator.
 *
 * cut_generator_jvp: deta[r][s] = sum_q (d eta_r / d h_q) dh[q][s] (double,
 * FP64 arithmetic): the quotient rule for CUT_GEN_G2 and CUT_GEN_G1 (d|eps|/d eps
 * = sign(eps), 0 at eps = 0), the product rule over the E_eta records for
 * CUT_GEN_WEGNER_GRAPH.  Errors as cut_generator. */
cut_status cut_generator_jvp(cut_graph_t g, int32_t kind, double delta, int64_t nsets,
                             const double* h, int64_t ldh, const double* dh, int64_t lddh,
                             double* deta, int64_t ldde, void* stream);

/* cut_graph_jvp: the directional derivative (Eq. directional-derivative)
 *   dy = apply(eta'(h) dh, x) + apply(eta(h), dx)
 * (the induced generator variation plus the linear response), and, when y is
 * not NULL, the action itself y = apply(eta(h), x).  Either tangent may be NULL
 * (a zero direction; not both); x may be NULL only when dh and y are.  All
 * pointers are double device memory; ld* are leading dimensions in elements
 * (ldh, lddh >= nsets; ldx, lddx, ldy, lddy >= nops*nsets).  The generator and
 * its derivative are FP64; the graph passes use `precision` (for the float
 * modes eta, eta'(h) dh, x and dx are rounded to float once).  Outputs are
 * overwritten and must not alias an input.  Uses the forward tiling of
 * cut_graph_set_tiling and the work area reserved with CUT_RESERVE_DERIV.
 * Errors: CUT_E_INVAL (also a shape that was not reserved), CUT_E_UNSUPPORTED
 * (G2 without a pair-flip registry), CUT_E_DEVICE. */
cut_status cut_graph_jvp(cut_graph_t g, int32_t kind, double delta, int32_t precision, int64_t nsets,
                         int64_t nops, const double* h, int64_t ldh, const double* dh, int64_t lddh,
                         const double* x, int64_t ldx, const double* dx, int64_t lddx, double* y,
                         int64_t ldy, double* dy, int64_t lddy, void* stream);

/* cut_graph_vjp: the transpose of cut_graph_jvp for a cotangent w of F
 * ([N][nops*nsets], double):
 *   g_x (=|+=) L(eta(h))^T w                     (records grouped by right input)
 *   g_h (=|+=) eta'(h)^T geta,  geta[i][s] = sum_{e: i_e=i} c_e sum_op w[k_e][op*nsets+s] x[j_e][op*nsets+s]
 * (records grouped by left input, then the generator VJP); `=|+=` follows
 * CUT_ACCUMULATE in flags.  Either output may be NULL (not both); x may be NULL
 * when g_h is.  Passes use `precision` (w, x and eta rounded to float once in
 * the float modes); the generator VJP is FP64.  Needs a graph loaded with
 * CUT_LOAD_ADJOINT.  Outputs must not alias an input.  Errors as cut_graph_jvp. */
cut_status cut_graph_vjp(cut_graph_t g, int32_t kind, double delta, int32_t precision, int64_t nsets,
                         int64_t nops, const double* h, int64_t ldh, const double* x, int64_t ldx,
                         const double* w, int64_t ldw, double* g_h, int64_t ldgh, double* g_x,
                         int64_t ldgx, uint32_t flags, void* stream);

/* --------------------------------------------------------------- assembly --
 * cut_assemble: output operators as linear combinations of a transformed
 * source library (Sec. 2.4, last paragraph; Sec. 3.4: one completed transform
 * serves many output combinations without another expansion):
 *   Y[n][k] (=|+=) sum_{s < S} X[n][s] * W[s][k],   0 <= n < N, 0 <= k < K,
 * X [N][ldx] the transformed coefficient vectors of the S sources (one column
 * per source, e.g. the operand columns of a flowed state), W [S][ldw] the
 * weights, Y [N][ldy]; all double, device memory owned by the caller; `=|+=`
 * follows CUT_ACCUMULATE.  FP64 on the matrix cores (MFMA 16x16x4 FP64; each
 * output is summed in chunks of 4 sources in source order).  Needs no graph.
 * Requires S >= 1, K >= 1, N >= 0, ldx >= S, ldw >= K, ldy >= K, K <= 4194240;
 * Y must not alias X or W.  Errors: CUT_E_INVAL, CUT_E_DEVICE. */
cut_status cut_assemble(const double* X, int64_t ldx, int64_t N, int64_t S, const double* W, int64_t ldw,
                        int64_t K, double* Y, int64_t ldy, uint32_t flags, void* stream);

/* ------------------------------------------------------------------- flow --
 * Coflow of H and nops-1 observables (Eq. coflow; Eq. forward-coeff) with the
 * classic fourth-order Runge-Kutta scheme at fixed step ds.  State z is double
 * [N][nops][nsets] (row-major, no padding), op 0 = H.  Set s advances while the
 * global step t satisfies t < n_steps[s], then stays frozen.  The generator,
 * the RK stage combination and the state are FP64; graph passes use
 * `precision` (operands are rounded to float once per stage for the float
 * modes).  Each RK step is one stream-ordered sequence of kernels; with
 * CUT_FLOW_HIPGRAPH it is captured once as a hipGraph and replayed. */
#define CUT_FLOW_HIPGRAPH 1u
#define CUT_FLOW_TIME_PASSES 2u  /* without CUT_FLOW_HIPGRAPH: bracket every graph
                                    pass and generator launch with HIP events on
                                    the launch stream (see cut_flow_last_timing);
                                    the call then synchronises to read them */

typedef struct {
    int32_t generator;      /* cut_generator_kind */
    int32_t precision;      /* cut_precision of the graph passes */
    double ds;              /* RK4 step */
    double delta;           /* G2 regulariser */
    int32_t ckpt_every;     /* checkpoint period in steps (0 = none) */
    uint32_t flags;         /* CUT_FLOW_HIPGRAPH */
    int64_t step_begin;     /* first global step to take (normally 0) */
    int64_t step_end;       /* one past the last step; < 0 = max(n_steps) */
    double* outside_norm2;  /* NULL, or device [nops*nsets] doubles: outside-space
                               diagnostic, see cut_flow_integrate */
    int32_t* nonfinite;     /* NULL: the call synchronises `stream` at its end and
                               returns CUT_E_NUMERIC if the result holds a
                               non-finite value.  Otherwise a device int32 that
                               the call sets to 0 at its start and to 1 if the
                               result holds a non-finite value; the call then
                               returns without synchronising. */
} cut_flow_params;

/* cut_flow_integrate: advances z in place over global steps [step_begin,
 * step_end).  n_steps is a HOST array of nsets int32.  If ckpt is not NULL and
 * ckpt_every > 0, slot c of ckpt (each N*nops*nsets doubles, device) receives z
 * at global step c*ckpt_every for every such step in range.
 * Outside-space diagnostic (Eq. projected-flow, C_X = (I - P)[eta, X], which
 * never feeds the flow): if outside_norm2 is not NULL the graph must hold E_C,
 * and every step a set takes adds sum_s b_s ds sum_q C_q(Z_s)^2 to
 * outside_norm2[op*nsets + s] (b = 1/6, 1/3, 1/3, 1/6, Z_s the RK stage states,
 * C the outside-space action with the stage generator, in the pass precision;
 * sums of squares in FP64, fixed order): the RK4 quadrature of the integral of
 * |C_X|^2 over the flow.  The flowed z is bitwise the same with or without it.
 * The work area must be reserved (CUT_RESERVE_FLOW) for (nsets, nops).
 * Errors: CUT_E_INVAL (also outside_norm2 without E_C, or a shape that was not
 * reserved), CUT_E_UNSUPPORTED (G2 on a non-Majorana graph), CUT_E_DEVICE,
 * CUT_E_NUMERIC (non-finite z after the flow, when nonfinite is NULL). */
cut_status cut_flow_integrate(cut_graph_t g, const cut_flow_params* p, int64_t nsets,
                              int64_t nops, const int32_t* n_steps, double* z, double* ckpt,
                              void* stream);

/* cut_flow_adjoint: exact adjoint of the discrete RK4 map (reverse-mode
 * gradient through the flow; graph-level adjoint of Sec. 2.4 plus the induced
 * generator variation of Eq. directional-derivative).  Needs the checkpoints of
 * a cut_flow_integrate call from step 0 with the same parameters, and a graph
 * loaded with CUT_LOAD_ADJOINT.  lambda (device, layout of z): in dL/dz at the
 * end of the flow, out dL/dz at step 0.  Each checkpoint block is recomputed
 * forward in FP64 with its stage states kept; all adjoint passes are FP64.
 * outside_norm2 is ignored; nonfinite as in cut_flow_integrate (checks lambda).
 * The work area must be reserved with CUT_RESERVE_ADJOINT for (nsets, nops,
 * ckpt_every). */
cut_status cut_flow_adjoint(cut_graph_t g, const cut_flow_params* p, int64_t nsets,
                            int64_t nops, const int32_t* n_steps, const double* ckpt,
                            double* lambda, void* stream);

/* ---------------------------------------------------------------- tuning --
 * Segment tiling of the graph passes.  Targets with more than `long_records`
 * records are "long".  Forward passes over E_L cut every long target into
 * chunks of about `chunk_records` records, one wavefront each, placed at their
 * relative position in the target so that the chunks running together sweep
 * the same operand region (for Majorana graphs every target's records are
 * ordered at load by the three modes its quartic operands share with the other
 * operand or the target, which makes that region small); the chunk sums are
 * kept as partial rows and added in chunk order.  Other passes split a long
 * target over the four wavefronts of a workgroup.  Shorter targets are packed
 * four to a workgroup, one per wavefront.
 * CUT_TILE_XCD_REMAP: consecutive chunk and task ranges run on one XCD (one L2).
 * CUT_TILE_NO_CHUNKS: no chunked form.
 * CUT_TILE_TRIPLE_CHUNKS (Majorana graphs): every quartic target K is also cut,
 * into chunks of whole shared-triple groups (the records whose quartic operand
 * is T+w for one triple T of K; about chunk_records records per chunk), placed
 * at the rank of T, so the chunks of all targets containing T run together and
 * read the rows T+w while they are in cache.
 * CUT_TILE_QUAD_BLOCKS (Majorana graphs, forward passes in the float modes with
 * nops <= 6): every quadratic target {u, v} pairs the rows T+u and T+v over all
 * triples T outside {u, v}; modes are grouped by 8, and one workgroup owns the
 * (up to 64) targets of two groups and a range of triples, stages the rows T+w
 * of its 16 modes in LDS once per triple and keeps its targets' sums in
 * registers; each (target, range) sum is a partial row added in fixed order.
 * CUT_TILE_TRIPLES (Majorana graphs, forward passes, nsets >= 8): every record
 * of a quartic target pairs a quadratic string with a quartic string sharing
 * three modes tau with the target; the 4-subsets containing tau are both the
 * targets and the quartic operands of those records, so they are staged in LDS
 * once per tile and each target's four tile sums are added in fixed order.
 * CUT_TILE_BCHUNK(b), b = 32, 16 or 8 (the B-chunk): the segment kernel's
 * forward passes give one record at most b lanes, one per coefficient set, so
 * a launch over more sets runs ceil(sets / b) workgroup columns, each reading
 * the record stream for its b sets (default, b = 64: one column for up to 64
 * sets).  Narrower lane groups hold more records per wavefront step; wider ones
 * read the records once for more sets.  The block and tile kernels keep their
 * own set blocking.
 * The chunked and tile forms need a work area of partial rows: the work areas
 * are re-sized for every shape reserved so far (cut_graph_reserve).  Rebuilds
 * the task lists of every loaded copy; synchronises the device.
 * Errors: CUT_E_INVAL (null handle, a length < 1, unknown flag), CUT_E_DEVICE. */
#define CUT_TILE_XCD_REMAP 1u
#define CUT_TILE_TRIPLES 2u
#define CUT_TILE_NO_CHUNKS 4u
#define CUT_TILE_TRIPLE_CHUNKS 8u
#define CUT_TILE_QUAD_BLOCKS 16u
#define CUT_TILE_BCHUNK_SHIFT 5    /* 2-bit field: B-chunk 64 >> field */
#define CUT_TILE_BCHUNK(b) ((uint32_t)((b) == 32 ? 1u : (b) == 16 ? 2u : (b) == 8 ? 3u : 0u) << CUT_TILE_BCHUNK_SHIFT)
cut_status cut_graph_set_tiling(cut_graph_t g, int64_t long_records, int64_t chunk_records, uint32_t flags);

/* Autotuner: times the forward graph pass for (nsets, nops) over candidate
 * tilings (chunk length 64/128/256/512 records, XCD remap off/on, triple
 * chunks, no chunks, shared-triple tiles and quadratic-target blocks where
 * available; long-target threshold 1024), then the three fastest of those with
 * the narrower B-chunks that the set count allows, and, when `precision` is CUT_F32C or
 * CUT_F32X and `allow_other_float` != 0, over both compensated float modes;
 * applies the fastest tiling to the graph (a candidate must beat the best so
 * far, starting with the graph's current tiling, by at least 2 %) and returns
 * the choice.  It allocates temporary operand buffers (zero-filled) and
 * synchronises the device.  Results are cached per (nsets, nops, precision,
 * allow_other_float).
 * Errors: CUT_E_INVAL, CUT_E_NOMEM, CUT_E_DEVICE. */
typedef struct {
    int64_t long_records;
    int64_t chunk_records;
    uint32_t tiling_flags;  /* CUT_TILE_* flags of the fastest configuration */
    int32_t precision;      /* fastest precision among the allowed ones */
    double pass_ms;         /* its average pass time */
    double default_ms;      /* time of the initial configuration */
} cut_tuning;
cut_status cut_graph_autotune(cut_graph_t g, int64_t nsets, int64_t nops, int32_t precision,
                              int32_t allow_other_float, cut_tuning* out);

/* Per-kernel timing of the last cut_flow_integrate call made with
 * CUT_FLOW_TIME_PASSES: summed HIP-event elapsed milliseconds and launch counts
 * of the fused graph passes and of the generator launches.  Zeros when the last
 * flow was not timed.  Errors: CUT_E_INVAL (null argument). */
typedef struct {
    double pass_ms;
    int64_t pass_launches;
    double gen_ms;
    int64_t gen_launches;
} cut_flow_timing;
cut_status cut_flow_last_timing(cut_graph_t g, cut_flow_timing* t);

const char* cut_last_error(void);
const char* cut_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CUTGRAPH_H */
