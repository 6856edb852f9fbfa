/*
 * efie.h -- C ABI of libefie, a gfx950 (MI355X) implementation of the dense
 * RWG-discretised electric field integral equation (EFIE) for PEC scatterers
 * and of the Calderon product preconditioner built on it.
 *
 * Formulation (readings of the paper where it is silent are listed per call):
 *   time factor e^{+j omega t}, Green's function G_k(R) = exp(-j k R)/(4 pi R)
 *     -- the convention fixed by the Hankel function H0^(2) of the paper's
 *        Green's function (Sec. II, eq. 5), carried to 3-D;
 *   Galerkin matrices (O)_mn = (f_m, O f_n) over RWG functions f_n
 *     -- the paper's operator-matrix notation of Sec. III with RWG as the basis;
 *   Z = eta (j k T_A + T_Phi/(j k)),  (T_A)_mn = <f_m, G f_n>,
 *   (T_Phi)_mn = <div f_m, G div f_n>,  Z J = V,  V_m = <f_m, E_inc>;
 *   Calderon product  T_BC(k~) Gmix^-1 Z(k)  with k~ = k - 0.4 j k^(1/3) a^(-2/3)
 *     -- the multiplicative structure and the complex wavenumber of the
 *        Calderon-stabilised operator of Sec. III.
 *
 * Conventions for every call:
 *   - Return value: efie_status.  0 = EFIE_OK, 1 = EFIE_NOT_CONVERGED (a warning:
 *     outputs are filled), < 0 = error; efie_last_error() then holds a message
 *     (thread-local, valid until the next call on the same thread).
 *   - No C++ exception crosses this boundary.
 *   - "dev" pointers are device memory owned by the caller (allocated e.g. by
 *     torch); the library never frees them and never allocates device memory
 *     except where a call says so.  "host" pointers are ordinary host memory.
 *   - Complex buffers are interleaved (re, im): complex128 = 2 doubles,
 *     complex64 = 2 floats.  Vectors and multi-vectors are row-major
 *     (nrhs, N): right-hand side s occupies N consecutive complex numbers.
 *   - Z is N x N row-major; it is symmetric (Z = Z^T), so rows and columns
 *     may be exchanged freely.
 *   - Device work is enqueued on the given stream; calls that return host
 *     values synchronise that stream before returning.  The workspace
 *     assemblies (efie_assemble_ws, the Calderon build) also run the near
 *     pairs of each chunk on a library-owned side stream of the current device
 *     (default priority, one per host thread), forked from and joined back to
 *     the given stream by events, so the call stays ordered on that stream.
 *   - Calls on one mesh handle are not thread-safe.
 */
#ifndef EFIE_H
#define EFIE_H

#include <stddef.h>
#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define EFIE_ABI_VERSION 1

typedef enum {
    EFIE_OK = 0,
    EFIE_NOT_CONVERGED = 1,
    EFIE_ERR_ARG = -1,              /* bad argument (null, size, range)            */
    EFIE_ERR_MESH_OPEN = -2,        /* an edge belongs to one triangle only        */
    EFIE_ERR_MESH_NONMANIFOLD = -3, /* an edge belongs to more than two triangles  */
    EFIE_ERR_MESH_ORIENT = -4,      /* neighbouring triangles oriented inconsistently */
    EFIE_ERR_DEGENERATE = -5,       /* zero-area triangle                           */
    EFIE_ERR_HIP = -6,              /* a HIP runtime call failed                    */
    EFIE_ERR_BREAKDOWN = -7,        /* Krylov breakdown (zero denominator)          */
    EFIE_ERR_NAN = -8,              /* NaN/Inf met in a residual                    */
    EFIE_ERR_STATE = -9             /* call order violated (e.g. tables not uploaded) */
} efie_status;

typedef enum { EFIE_C128 = 0, EFIE_C64 = 1 } efie_dtype;
typedef enum { EFIE_COCG = 0, EFIE_CGS = 1 } efie_solver;

typedef struct efie_mesh_s* efie_mesh;

/* Library version of this header's ABI. */
int efie_abi_version(void);

/* Message of the last failing call on this thread ("" if none). */
const char* efie_last_error(void);

/* ------------------------------------------------------------------ mesh */

/*
 * Build the RWG topology of a closed, consistently oriented triangle mesh
 * (outward normals, counter-clockwise vertex order seen from outside).
 *   xyz  host, nv x 3 doubles (metres);  tri host, nt x 3 vertex ids.
 *   near_factor > 0: triangle pairs that share a vertex or whose centroid
 *   distance is below near_factor * max(longest edge of either) are "near"
 *   and get singularity extraction (reading: the paper gives no near rule).
 * RWG numbering: interior edges (a, b), a < b, in lexicographic order; T+ is the
 * triangle whose boundary runs a -> b, T- the one running b -> a (RWG 1982).
 * Errors: EFIE_ERR_ARG, EFIE_ERR_MESH_*, EFIE_ERR_DEGENERATE.  *out is set
 * only on success; release it with efie_mesh_destroy.
 */
int efie_mesh_create(const double* xyz, int64_t nv, const int32_t* tri, int64_t nt,
                     double near_factor, efie_mesh* out);

void efie_mesh_destroy(efie_mesh mesh);

/*
 * Distance-adaptive far rule (not in the paper; off by default).  With
 * ratio > 0, a far triangle pair (not near) whose centroid distance D satisfies
 * D^2 >= (ratio * h)^2, h the larger longest edge of the two triangles (FP64,
 * no fused operations), is integrated with the 3x3 product of the interior
 * 3-point degree-2 rule (barycentric (2/3, 1/6, 1/6) and permutations, equal
 * weights; Strang and Fix 1973) instead of the 7x7 rule: 9 Green's-function
 * evaluations instead of 49.  ratio = 0 restores the 7x7 rule everywhere.
 * Applies to every later assembly of this mesh (efie_assemble, efie_assemble_ws,
 * and the barycentric operator of an efie_calderon created from it, whose pairs
 * are measured in their own triangles' edges, unless efie_calderon_set_far_rule
 * gives that operator a rule of its own); efie_batch_* and
 * efie_vertex_grad reject a mesh with the rule on (EFIE_ERR_ARG).  Accuracy: the
 * 3x3 rule's error on a pair falls as (h / D)^3 and (k h)^3; on a level-2
 * sphere (ratio 3, k = 1) Z moves by 2e-5 (Frobenius, relative) and the RCS by
 * under 0.01 dB.  Errors: EFIE_ERR_ARG (null mesh, ratio < 0 or not finite).
 */
int efie_mesh_set_far_rule(efie_mesh mesh, double ratio);

/*
 * Largest |Re k| accepted by the complex64 assemblies of this mesh (efie_assemble
 * and efie_assemble_ws with EFIE_C64, the complex64 barycentric pairs of
 * efie_calderon_assemble_ex, efie_batch_assemble with EFIE_C64).  Their FP32
 * far-pair kernels hand the phase Re(k) R, in revolutions, to the hardware sine
 * and cosine, whose argument must stay below 256 revolutions; R never exceeds the
 * bounding-box diagonal D of the vertices, so the limit is 512 pi / D.  Those
 * calls return EFIE_ERR_ARG at or beyond it, before any device work (EFIE_C128
 * has no such limit).  Host only.  Errors: EFIE_ERR_ARG (null argument).
 */
int efie_mesh_fp32_kmax(efie_mesh mesh, double* kmax);

/* Sizes: RWG count N, triangle count T, ordered near pairs (incl. self pairs),
 * and the byte size of the device tables required by efie_mesh_upload. */
int efie_mesh_sizes(efie_mesh mesh, int64_t* n_rwg, int64_t* n_tri, int64_t* n_near,
                    size_t* table_bytes);

/* Host copy of the numbering: edge_v (N x 2 vertex ids a < b), edge_t (N x 2:
 * T+, T-).  Either pointer may be NULL. */
int efie_mesh_rwg_table(efie_mesh mesh, int32_t* edge_v, int32_t* edge_t);

/* Copy the structure-of-arrays geometry tables into dev (table_bytes bytes,
 * 256-byte aligned, caller-owned, must outlive every later call on the mesh).
 * Synchronises the stream. */
int efie_mesh_upload(efie_mesh mesh, void* dev, size_t bytes, hipStream_t stream);

/* -------------------------------------------------------------- assembly */

/*
 * Z = eta (j k T_A + T_Phi/(j k)) for complex k = k_re + j k_im (k_im <= 0),
 * 7-point degree-5 rule per triangle (reading: the paper names no rule), 7x7
 * product rule per triangle pair; near pairs split G into (exp(-jkR)-1)/(4 pi R)
 * (same rule; -jk/(4 pi) at R = 0) plus 1/(4 pi R), the latter with the
 * closed-form inner integrals of Wilton et al. 1984 / Graglia 1993 over the
 * source triangle and the 7-point rule over the test triangle, averaged with
 * its transpose so that Z is exactly symmetric (reading).
 *   Z dev, N x N complex of type dtype.
 *   EFIE_C128: every pair in FP64.
 *   EFIE_C64 : far pairs in FP32 arithmetic, near pairs in FP64, stored as complex64.
 * parts != 0 returns T_A in Z and T_Phi in Z2 (dev, same shape) instead of Z
 * (eta and k then only enter the Green's function); otherwise Z2 is ignored.
 */
int efie_assemble(efie_mesh mesh, double k_re, double k_im, double eta, int dtype,
                  void* Z, void* Z2, int parts, hipStream_t stream);

/*
 * The same Z as efie_assemble (parts = 0) without atomics: the pair values of the
 * triangle pairs with source triangle q >= p (q = p halved) are written per chunk
 * of test triangles into the caller's workspace and added row by row into U, and
 * Z = U + U^T by mirror tiles, so the result is deterministic (bit-identical
 * between runs) and exactly symmetric.  Any
 * ws_bytes >= min_bytes works (chunks of ws_bytes / min_bytes test triangles);
 * full_bytes (= T x min_bytes) holds all triangles in one chunk.
 *   min_bytes = 6 N x (16 for EFIE_C128, 8 for EFIE_C64);  ws dev, 16-byte aligned.
 * Errors: EFIE_ERR_ARG if ws_bytes < min_bytes.
 */
int efie_assemble_workspace_size(efie_mesh mesh, int dtype, size_t* min_bytes, size_t* full_bytes);
int efie_assemble_ws(efie_mesh mesh, double k_re, double k_im, double eta, int dtype, void* Z,
                     void* ws, size_t ws_bytes, hipStream_t stream);

/* ------------------------------------------------------------ excitation */

/*
 * V[s][m] = int f_m . E0 pol_s exp(-j k khat_s . r) dS by the 7-point rule.
 *   khat, pol dev, nrhs x 3 doubles (unit propagation vector, polarisation);
 *   V dev, nrhs x N complex128.
 */
int efie_excite_planewave(efie_mesh mesh, double k, const double* khat, const double* pol,
                          int64_t nrhs, double e0, void* V, hipStream_t stream);

/* --------------------------------------------------------------- far field */

/*
 * Far-field pattern F(rhat) = -(j k eta/4 pi) (I - rhat rhat) . sum_n J_n
 * int f_n exp(j k rhat . r') dS' (7-point rule), in (theta-hat, phi-hat)
 * components; RCS = 4 pi |F|^2 / |E0|^2.
 *   J dev (nrhs, N) complex128;  dirs dev (ndir, 3) unit vectors;
 *   F dev (nrhs, ndir, 2) complex128.
 *   ws dev workspace of at least efie_farfield_workspace_size bytes.
 */
int efie_farfield_workspace_size(efie_mesh mesh, int64_t ndir, size_t* bytes);
int efie_farfield(efie_mesh mesh, double k, double eta, const void* J, int64_t nrhs,
                  const double* dirs, int64_t ndir, void* F, void* ws, size_t ws_bytes,
                  hipStream_t stream);

/*
 * Adjoint source of the far field: G[s][n] = sum_{d,c} W[s][d][c] R_dc,n with
 * R_dc,n = -(j k eta/4 pi) e_c(rhat_d) . int f_n exp(j k rhat_d . r') dS', the
 * matrix that maps a current to its far field (F = R J).  With W = conj(F) this
 * is dJ/dJ^T of J = sum |F|^2, the right-hand side of the adjoint solve
 * Z lambda = G (Z = Z^T).
 *   W dev (nrhs, ndir, 2) complex128;  dirs dev (ndir, 3);  G dev (nrhs, N)
 *   complex128;  ws as for efie_farfield (same size).
 */
int efie_farfield_adjoint(efie_mesh mesh, double k, double eta, const void* W, int64_t nrhs,
                          const double* dirs, int64_t ndir, void* G, void* ws, size_t ws_bytes,
                          hipStream_t stream);

/*
 * The far-field objective of the differentiation form and its adjoint weight:
 * J = sum_i |F_i|^2 over the count complex far-field values F (e.g. the
 * (nrhs, ndir, 2) output of efie_farfield), and W = conj(F), the derivative of J
 * with respect to F that efie_farfield_adjoint and efie_vertex_grad take.
 *   F dev complex128 (count);  J dev, one double (written);  W dev complex128
 *   (count, written) or NULL;  W must not alias F.  The sum runs in a fixed order
 *   (the same value on every call).  Errors: EFIE_ERR_ARG (null F or J,
 *   count < 1, W == F).
 */
int efie_farfield_objective(const void* F, int64_t count, void* J, void* W, hipStream_t stream);

/* -------------------------------------------------------- vertex gradient */

/*
 * Gradient with respect to the vertex positions of an objective J(F) of the far
 * field F = R(x) J of the solution of Z(x) J = V(x), for one right-hand side
 * (plane wave khat, pol, e0) -- the shape-derivative use of the discretised
 * operator (the EFIE of Sec. II with the matrices of Sec. III as functions of
 * the mesh vertices x).  Given J, the adjoint lambda (Z lambda = R^T W) and
 * W = dJ/dF (W = conj(F) for J = sum |F|^2), it returns
 *   dxyz = 2 Re[ W^T (dR/dx) J + lambda^T (dV/dx) - lambda^T (dZ/dx) J ].
 * Z is the k-real operator of efie_assemble (same quadrature, near rule frozen
 * at the mesh's current classification, singular parts symmetrised).  Far pairs
 * are differentiated analytically, near pairs by forward-mode dual numbers
 * through the smooth part and the closed-form singular integrals.  FP64.
 *   J, lambda dev (N) complex128;  W dev (ndir, 2) complex128;  dirs dev
 *   (ndir, 3);  khat, pol host 3 doubles;  dxyz dev (nv, 3) doubles
 *   (overwritten);  ws dev, efie_vertex_grad_workspace_size bytes (T x 9
 *   doubles).  Asynchronous on stream.
 */
int efie_vertex_grad_workspace_size(efie_mesh mesh, size_t* bytes);
int efie_vertex_grad(efie_mesh mesh, double k, double eta, const void* J, const void* lambda,
                     const void* W, const double* dirs, int64_t ndir, const double* khat,
                     const double* pol, double e0, double* dxyz, void* ws, size_t ws_bytes,
                     hipStream_t stream);

/* ----------------------------------------------------------- Z . X products */

/*
 * Y = Z X for a dense complex matrix Z (n x n, row-major, either dtype) and
 * nrhs vectors X (nrhs, n).  X and Y have the dtype of Z.
 *   nrhs == 1: HBM-bound GEMV (accumulation in FP64 for both dtypes);
 *   nrhs > 1 : EFIE_C64 -> FP32 matrix-core (MFMA) GEMM with FP32 accumulation,
 *              EFIE_C128 -> FP64 GEMM.
 */
int efie_zx(const void* Z, int dtype, int64_t n, const void* X, void* Y, int64_t nrhs,
            hipStream_t stream);

/*
 * The mixed solves' product as a call of its own: Y = Z X with Z complex64
 * (n x n) and X, Y complex128 (nrhs, n).  X is rounded to complex64 and
 * multiplied on the FP32 matrix cores with the partial sums of every two K
 * chunks (at most 64 complex terms) flushed into FP64 accumulators; Y is
 * written in complex128.  Any nrhs >= 1
 * takes the matrix cores here.  ws: dev scratch of at least
 * efie_zx_flush64_workspace_size bytes, 16-byte aligned.  Y must not overlap X.
 */
int efie_zx_flush64_workspace_size(int64_t n, int64_t nrhs, size_t* bytes);
int efie_zx_flush64(const void* Z, int64_t n, const void* X, void* Y, int64_t nrhs, void* ws,
                    size_t ws_bytes, hipStream_t stream);

/*
 * efie_zx_flush64 for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product and the same kernels, with the complex64 copy of X and the row list
 * kept in a library-owned scratch array of 64 MiB per GPU (a static device
 * array, one copy on each device the library runs on, held until the process
 * ends) instead of a caller workspace.  Allocates nothing and calls no allocating
 * routine.  Limit: n * nrhs * 8 bytes, rounded up to a multiple of 256, plus
 * 4 * nrhs bytes must not exceed the scratch (efie_zx_flush64_noalloc_max gives
 * its size; e.g. n = 30720 with nrhs <= 273); larger products return EFIE_ERR_ARG.
 * Every call on one GPU shares that GPU's scratch: calls that overlap on one GPU
 * (two streams, or two host threads without ordering) race and give wrong
 * results; calls ordered on one stream are safe.  Every scratch element a call
 * reads is written earlier in the same call.  Z, X, Y, n, nrhs as for
 * efie_zx_flush64; asynchronous on stream.
 */
int efie_zx_flush64_noalloc_max(int64_t* max_bytes);
int efie_zx_flush64_noalloc(const void* Z, int64_t n, const void* X, void* Y, int64_t nrhs, hipStream_t stream);

/* ------------------------------------------------------- GEMM autotuning */

/*
 * The complex64 matrix-core GEMM has several tile shapes (block tile of BM
 * right-hand sides x BN unknowns, K chunk KC of complex elements), for two
 * paths: complex64
 * output (efie_zx) and FP64-flushed output into the Krylov vectors (solves).
 * efie_gemm_autotune times every variant on the caller's Z (n x n complex64) and
 * X (M x n complex64) with HIP events (reps launches each, after one warm-up),
 * writes the mean milliseconds per launch into ms[variant] (host, count
 * entries), returns in *best the first variant (in table order) within 2 % of
 * the fastest, so that timing noise does not flip between near-equal tiles, and
 * does not change the selection.
 * ws: dev scratch of at least M*n*(acc64 ? 16 : 8) bytes rounded up to 256, plus
 * 4*M bytes.  efie_gemm_select sets the variant used by later calls (process-wide).
 */
int efie_gemm_variants(int* count);
int efie_gemm_variant_info(int variant, int* bm, int* bn, int* kc);
int efie_gemm_autotune(const void* Z, int64_t n, const void* X, int64_t M, int acc64, void* ws,
                       size_t ws_bytes, int reps, double* ms, int* best, hipStream_t stream);
int efie_gemm_select(int acc64, int variant, int* previous);

/*
 * The autotuner with a persistent cache of its choices.  For a Z of order n
 * (complex64, dev) times M right-hand sides on the current device, the cache
 * file cache_path (plain text, one line per entry: a key naming the device, n, M
 * and the tile table, the chosen variants of the complex64-output and the
 * FP64-flush paths, and the mean milliseconds of every variant on each path) is
 * read; an entry with the same key is reused unless force != 0.  Otherwise both
 * paths are timed as by efie_gemm_autotune (reps launches after a warm-up) on a
 * seeded block X generated on the device, and the entry is added (the file is
 * rewritten through a temporary file and a rename; an unwritable file leaves the
 * result valid).  Either way both variants are selected as by efie_gemm_select.
 * cache_path may be NULL (always time, keep nothing).  Outputs (host):
 * variant_acc32, variant_acc64; ms_acc32 / ms_acc64 (efie_gemm_variants entries
 * each, may be NULL); from_cache (may be NULL) = 1 when the entry was reused.
 * ws: dev, 256-byte aligned, efie_gemm_autotune_cached_workspace_size bytes.
 * Synchronises the stream when it times.  Malformed cache lines are ignored and
 * dropped when the file is rewritten.
 */
int efie_gemm_autotune_cached_workspace_size(int64_t n, int64_t M, size_t* bytes);
int efie_gemm_autotune_cached(const char* cache_path, const void* Z, int64_t n, int64_t M, int reps, int force,
                              void* ws, size_t ws_bytes, int* variant_acc32, int* variant_acc64, double* ms_acc32,
                              double* ms_acc64, int* from_cache, hipStream_t stream);

/* ------------------------------------------------------------------ solve */

typedef struct {
    int32_t solver;       /* EFIE_COCG (default) or EFIE_CGS                         */
    int32_t maxit;        /* iteration cap of one Krylov solve                       */
    double tol;           /* target ||V - Z J||_2 / ||V||_2 per right-hand side      */
    int32_t max_refine;   /* EFIE_C64 only: outer refinement steps (>= 1)            */
    double inner_tol;     /* EFIE_C64 only: relative tolerance of each inner solve   */
    int32_t fp32_acc;     /* EFIE_C64 only: 0 (default) = flush the FP32 matrix-core */
                          /* partial sums into FP64 every two K chunks; 1 = accumu-  */
                          /* late in FP32 (more Krylov iterations)                   */
} efie_solve_opts;

typedef struct {
    int32_t iters;        /* Krylov iterations (summed over refinement steps)        */
    int32_t status;       /* EFIE_OK, EFIE_NOT_CONVERGED or an error code             */
    double relres_recur;  /* last recurrence residual of the (last inner) solve       */
    double relres_true;   /* ||V - Z J|| / ||V|| recomputed at exit (FP64 accumulation) */
} efie_rhs_stats;

/*
 * Solve Z J = V for nrhs right-hand sides, x0 = 0 (readings: the paper names CG
 * and CGS without stating them; "CG" is COCG, CG with the unconjugated bilinear
 * form, valid since Z = Z^T; CGS is Sonneveld's with shadow residual r0).
 *   Z dev (dtype as assembled), V dev (nrhs, N) complex128, J dev (nrhs, N)
 *   complex128 (output).  FP64 vectors and inner products in both cases.
 *   EFIE_C128: one Krylov solve with FP64 products.
 *   EFIE_C64 : mixed precision -- Z X products of more than 8 active columns run
 *              on FP32 matrix cores with FP64 accumulation of the K-chunk partial
 *              sums (opts->fp32_acc = 1: FP32 accumulation); COCG replaces its recursive residual by the true residual
 *              V - Z J (FP64 accumulation from the stored complex64 Z) whenever it
 *              has dropped tenfold (reliable updates) and converges only on it;
 *              CGS runs inner solves to inner_tol inside an outer refinement loop
 *              (max_refine steps) on the same true residual.
 *   stats host, nrhs entries (may be NULL).
 *   ws dev workspace of efie_solve_workspace_size bytes.
 * Returns EFIE_NOT_CONVERGED if any right-hand side missed tol or broke down
 * (per-column EFIE_ERR_BREAKDOWN / EFIE_ERR_NAN in stats[s].status); negative
 * return codes are reserved for argument and HIP errors.  Synchronises.
 */
int efie_solve_workspace_size(int64_t n, int64_t nrhs, int dtype, size_t* bytes);
int efie_solve(const void* Z, int dtype, int64_t n, const void* V, void* J, int64_t nrhs,
               const efie_solve_opts* opts, efie_rhs_stats* stats, void* ws, size_t ws_bytes,
               hipStream_t stream);

/* --------------------------------------------------------------- Calderon */

/*
 * Calderon preconditioner of the EFIE (the paper's Sec. III, eq. 16 structure:
 * second operator at the complex wavenumber k~ = k - 0.4 j k^(1/3) a^(-2/3),
 * times a Gram inverse, times the first operator).  Readings for 3-D: the second
 * operator is the EFIE on Buffa-Christiansen functions g_n built on the
 * barycentric refinement (equal charge per barycentric triangle of each dual cell,
 * no flux across the primal edge), T_BC(k~) = R^T T_bary(k~) R with
 * g_n = sum_e R[e][n] f_e over barycentric RWGs; the Gram matrix is the mixed
 * (G_mix)_mn = int (n x f_m) . g_n dS.  The preconditioned system is
 * P Z J = P V with P = T_BC(k~) G_mix^-1 (dense, complex128, N x N).
 *
 * efie_calderon_create: host refinement, R and G_mix for a mesh (kept alive by
 *   the caller).  efie_calderon_upload: like efie_mesh_upload, table_bytes from
 *   efie_calderon_sizes.
 * efie_calderon_host_matrices: dense host copies (R: N_bary x N, G: N x N, either
 *   may be NULL) for inspection of small meshes.
 * efie_calderon_assemble: P into dev P (N x N complex128); optionally T_BC into
 *   dev Tbc_out (may be NULL).  T_BC is accumulated without forming T_bary: the
 *   barycentric pair values of a chunk of test triangles go to workspace rows
 *   (at most 2 GiB) that are contracted with R at once.  Rows of P solve
 *   G_mix^T p = T_BC row by BiCGStab (batches of rows, column layout) to the
 *   relative residual tol (maxit steps); *relres (host, may be NULL) gets the worst
 *   achieved.  For tol >= 1e-4 the solver's vectors are stored in complex64 (every
 *   sum, norm and update still in FP64), which bounds the attainable residual
 *   near 1e-6; tighter tolerances keep them in complex128.  ws: dev workspace of ws_bytes from efie_calderon_sizes (T_BC,
 *   16 N^2 bytes, plus a few GiB).  EFIE_NOT_CONVERGED if tol missed.
 * efie_calderon_assemble_ex: the same with bary_dtype EFIE_C128 (as above) or
 *   EFIE_C64: barycentric far pairs in FP32 (near pairs FP64) and complex64
 *   workspace rows; contractions, T_BC and P stay FP64 (a preconditioner only
 *   has to be fixed, not exact: P then differs from T_BC G^-1 by ~1e-6).
 * efie_solve_precond: CGS on P Z J = P V (complex128 Z and P, FP64 throughout).
 *   efie_solve_precond_ex: Z and P of either dtype; with a complex64 factor the
 *   CGS products of more than 8 columns run on FP32 matrix cores (FP64 flushes)
 *   and each pass stops no lower than opts->inner_tol, the outer refinement
 *   (FP64 products, against the stored Z) making the result accurate.  CGS
 *   tests the preconditioned recurrence residual; an outer refinement on the
 *   unpreconditioned FP64 true residual r = V - Z J then solves P Z d = P r for the
 *   columns still above tol (tolerance scaled by the observed ratio of true to
 *   preconditioned reduction) and adds d, up to opts->max_refine passes (>= 1).
 *   A column is EFIE_OK when ||V - Z J|| <= tol ||V||; stats report that residual
 *   and the CGS iterations summed over the passes.
 */
/*
 * The complex wavenumber of the Calderon second operator (Sec. III, the
 * definition that follows the preconditioned operator of eq. 16):
 *   k~ = k - 0.4 j k^(1/3) a^(-2/3),
 * a an average radius of curvature of the scatterer (a = 1 for the unit
 * sphere).  Host only.  Errors: EFIE_ERR_ARG (null output, k or a not finite
 * and > 0).
 */
int efie_ktilde(double k, double a, double* kt_re, double* kt_im);

typedef struct efie_calderon_s* efie_calderon;
int efie_calderon_create(efie_mesh mesh, efie_calderon* out);
void efie_calderon_destroy(efie_calderon c);
/* The far rule of the barycentric operator T_bary(k~) alone (see
 * efie_mesh_set_far_rule): ratio >= 0 sets it for later efie_calderon_assemble
 * calls, independently of the primal mesh; ratio < 0 (the default) makes it
 * follow the primal mesh's rule.  P only has to be a fixed approximation of
 * T_BC G_mix^-1, so a coarser rule here leaves the solution of P Z J = P V to
 * the accuracy of Z.  Errors: EFIE_ERR_ARG (null handle, ratio not finite). */
int efie_calderon_set_far_rule(efie_calderon c, double ratio);
int efie_calderon_sizes(efie_calderon c, int64_t* n_bary_rwg, int64_t* n_bary_tri, size_t* table_bytes,
                        size_t* ws_bytes);
int efie_calderon_upload(efie_calderon c, void* dev, size_t bytes, hipStream_t stream);
int efie_calderon_host_matrices(efie_calderon c, double* R, double* G);
int efie_calderon_assemble(efie_calderon c, double kt_re, double kt_im, double eta, void* P, void* Tbc_out,
                           double tol, int32_t maxit, double* relres, void* ws, size_t ws_bytes,
                           hipStream_t stream);
int efie_calderon_assemble_ex(efie_calderon c, double kt_re, double kt_im, double eta, int bary_dtype, void* P,
                              void* Tbc_out, double tol, int32_t maxit, double* relres, void* ws,
                              size_t ws_bytes, hipStream_t stream);
int efie_solve_precond_workspace_size(int64_t n, int64_t nrhs, size_t* bytes);
int efie_solve_precond(const void* Z, const void* P, int64_t n, const void* V, void* J, int64_t nrhs,
                       const efie_solve_opts* opts, efie_rhs_stats* stats, void* ws, size_t ws_bytes,
                       hipStream_t stream);
int efie_solve_precond_ex(const void* Z, int zdt, const void* P, int pdt, int64_t n, const void* V, void* J,
                          int64_t nrhs, const efie_solve_opts* opts, efie_rhs_stats* stats, void* ws,
                          size_t ws_bytes, hipStream_t stream);

/* --------------------------------------- Calderon-stabilized CFIE (3-D) */

/*
 * The paper's stabilized operator (Sec. III, eq. 16) adds to the Calderon product
 * of the electric operator that of the magnetic one (the MFIE part of the CFIE of
 * eq. 7), each second factor at k~.  In 3-D, with f RWG and g BC functions:
 *   K J = n x p.v. int grad G_k(r, r') x J(r') dS'   (MFIE: (1/2 - K) J = n x H^inc),
 *   K_BC(k)[m][n] = (g_m, p.v. int grad G_k x f_n dS')  (the MFIE tested with n x g_m),
 *   M  = eta (-G_mix^T / 2 - K_BC(k))     = eta (n x g_m, (1/2 - K_k) f_n),
 *   M~ = eta (-G_mix^T / 2 + K_BC(k~))    = eta (n x g_m, (1/2 + K_k~) f_n),
 *   Q  = M~ G_mix^-T,
 *   eta^2 C_p = P Z + Q M,   eta^2 b_p = P V + Q H,
 *   H[s][m] = (g_m, (khat_s x pol_s) exp(-j k khat_s . r)) = eta (g_m, H^inc_s)
 * with P = T_BC(k~) G_mix^-1 (efie_calderon_assemble) and Z, V the EFIE matrix and
 * right-hand side.  C_p is a second-kind operator (near -1/2 + 2 K~ K), free of the
 * interior resonances of the EFIE and of the MFIE.  The sign of the combination
 * follows from the Calderon identity (n x T/eta)^2 = -1/4 + K^2.
 * K_BC is built as R^T K_mix, K_mix[e][n] = (f_e, p.v. int grad G x f_n) over the
 * barycentric RWGs f_e (test triangle b inside primal triangle b / 6): zero on
 * the coplanar pair (b / 6, b / 6); singularity extraction (7-point smooth part
 * plus the closed-form int (r - r')/R^3 dS') on the primal pairs the EFIE near
 * rule calls near; the 7 x 7 product rule elsewhere.  FP64 throughout.
 *
 * efie_calderon_cfie_assemble: M and Q into dev buffers (N x N complex128 each),
 *   optionally K_BC(k) and K_BC(k~) (raw, N x N complex128) into K_out, Kt_out;
 *   k > 0 real, kt_im <= 0; Q by BiCGStab on G_mix to tol (maxit steps; complex64
 *   vectors when tol >= 1e-4), its worst relative residual in *relres.  Needs the
 *   mesh and the Calderon tables uploaded; ws as for efie_calderon_assemble
 *   (ws_bytes from efie_calderon_sizes).  Returns EFIE_NOT_CONVERGED if Q missed tol.
 * efie_calderon_mfie_rhs: H (dev, nrhs x N complex128) for the plane waves khat_s,
 *   pol_s (dev, nrhs x 3 doubles each); ws (256-aligned) of the size from
 *   efie_calderon_mfie_rhs_workspace_size.
 * efie_solve_cfie: CGS (opts->solver EFIE_CGS) on (P Z + Q M) J = P V + Q H, every
 *   matrix complex128 (n x n), V, H, J (nrhs x n); FP64 products; stats report the
 *   FP64 true residual of the stabilized system; ws from
 *   efie_solve_cfie_workspace_size.
 */
int efie_calderon_cfie_assemble(efie_calderon c, double k, double kt_re, double kt_im, double eta, void* M, void* Q,
                                void* K_out, void* Kt_out, double tol, int32_t maxit, double* relres, void* ws,
                                size_t ws_bytes, hipStream_t stream);
int efie_calderon_mfie_rhs_workspace_size(efie_calderon c, int64_t nrhs, size_t* bytes);
int efie_calderon_mfie_rhs(efie_calderon c, double k, const double* khat, const double* pol, int64_t nrhs, void* H,
                           void* ws, size_t ws_bytes, hipStream_t stream);
int efie_solve_cfie_workspace_size(int64_t n, int64_t nrhs, size_t* bytes);
int efie_solve_cfie(const void* Z, const void* P, const void* M, const void* Q, int64_t n, const void* V,
                    const void* H, void* J, int64_t nrhs, const efie_solve_opts* opts, efie_rhs_stats* stats,
                    void* ws, size_t ws_bytes, hipStream_t stream);

/* ---------------------------------------------------------- many meshes */

/*
 * A batch of uploaded meshes (uneven sizes) assembled together and solved
 * together (one right-hand side per mesh).
 * Layout: the Z of mesh i (caller order) occupies N_i^2 consecutive complex
 * elements of Zcat starting at sum_{j<i} N_j^2 (row-major, as efie_assemble);
 * vectors occupy N_i consecutive complex128 elements of Vcat / Jcat starting at
 * sum_{j<i} N_j.
 * efie_batch_create: meshes must stay alive.  efie_batch_sizes: table_bytes for
 *   efie_batch_upload (the Z and vector offsets and every mesh table concatenated
 *   over the meshes), ws_bytes for assemble/solve (with every mesh's near-pair
 *   blocks), total Z and vector elements, and the work items of the persistent
 *   assembly launch (the complex64 tiles of all meshes).
 * efie_batch_upload: copies the meshes' tables as they are at that call; the
 *   far-rule ratio of each mesh is read at each assemble.
 * efie_batch_assemble: k host array (nmesh, real, > 0); the tile assembly of
 *   efie_assemble_ws for every mesh in two launches: the near-pair blocks of all
 *   meshes, then one persistent launch over the tiles of all meshes' Z (a block per
 *   resident slot, tile t to block t mod grid): every Z bit-identical to
 *   efie_assemble_ws of its mesh, no atomics.  Synchronises.
 * efie_batch_solve: COCG per mesh (FP64 vectors), one grouped GEMV launch (FP64
 *   accumulation) and one grouped update launch per iteration; stats host nmesh.
 *   Per-mesh failures give EFIE_NOT_CONVERGED with the status in stats.
 */
typedef struct efie_batch_s* efie_batch;
int efie_batch_create(const efie_mesh* meshes, int32_t nmesh, efie_batch* out);
void efie_batch_destroy(efie_batch b);
int efie_batch_sizes(efie_batch b, size_t* table_bytes, size_t* ws_bytes, int64_t* z_elems, int64_t* v_elems,
                     int64_t* items);
int efie_batch_upload(efie_batch b, void* dev, size_t bytes, hipStream_t stream);
int efie_batch_assemble(efie_batch b, const double* k, double eta, int dtype, void* Zcat, void* ws,
                        size_t ws_bytes, hipStream_t stream);
int efie_batch_solve(efie_batch b, const void* Zcat, int dtype, const void* Vcat, void* Jcat,
                     const efie_solve_opts* opts, efie_rhs_stats* stats, void* ws, size_t ws_bytes,
                     hipStream_t stream);

/* ------------------------------------------------ the paper's 2-D method */

/*
 * The paper's own method on a closed curve (Sec. II-III): the boundary integral
 * operators of eqs. 1-5 with G_k(R) = -(j/4) H0^(2)(k R), discretized by
 * Galerkin with piecewise-linear functions on the polygon through the nodes, the
 * TM CFIE of a PEC cylinder (eq. 7, first row), its Calderon-stabilized form
 *   C_p = N_k~ G^-1 S_k + (G/2 - D*_k~) G^-1 (G/2 + D*_k)            (eq. 16)
 * and the fast direct solver: C_p = C_p,c + C_p,ext with C_p,c the circular
 * counterpart (C_p on a circle with the same node count, circulant), a skeleton
 * C_p,ext ~ U V^T from an adaptive randomized range finder, and
 *   C_p^-1 = C_c^-1 - C_c^-1 U (I + V^T C_c^-1 U)^-1 V^T C_c^-1      (eqs. 17-18).
 * Readings (the paper names none of them): Maue's form of N,
 *   (lambda_i, N lambda_j) = int int G [lambda_i' lambda_j' - k^2 (n.n') lambda_i lambda_j];
 * q x q Gauss-Legendre on segment pairs that share no node, a graded Duffy rule
 * (8 x 8 per triangle) on adjacent pairs, the self pair's log part in closed form;
 * TM excitation E_z = exp(-j k khat . r), khat = (cos phi, sin phi),
 * e_i = (lambda_i, E_z), h_i = (lambda_i, H_t) with H_t = -(khat . n) E_z / eta, and
 *   b_p = N_k~ G^-1 e/(j k eta) + (G/2 - D*_k~) G^-1 h;
 * the range finder samples blocks of a caller-given test matrix, projects each
 * twice against the basis so far and stops when its largest column norm is at
 * most tol times that of C_p Omega_0 (the first block applied to C_p).
 * Vectors are rows: (count, n) complex128, row-major.  All arithmetic FP64, the
 * dense products on FP64 matrix cores.
 *
 * efie_bie2d_create: nodes and circle_nodes host (n x 2), counter-clockwise (node
 *   i of the circle is the counterpart of node i of the curve); q = 2..6 or 8
 *   Gauss points per segment.  Errors: EFIE_ERR_ARG, EFIE_ERR_DEGENERATE (zero-length
 *   segment), EFIE_ERR_MESH_ORIENT (clockwise contour).
 * efie_bie2d_sizes: table_bytes for efie_bie2d_upload; ws_bytes of the workspace of
 *   efie_bie2d_setup for a skeleton of rank <= rmax, blocks of `block` columns
 *   (<= 64) and up to nvec vectors per call (nvec >= block).  The workspace holds
 *   S_k, D*_k, N_k~, D*_k~ (4 n^2 complex128) and the skeleton's factors.
 * efie_bie2d_assemble: a window [row0, row0 + nrows) x [col0, col0 + ncols) of
 *   S_k, D*_k and N_k of contour `which` (0 the curve, 1 the circle) into the
 *   non-null outputs (dev, row-major with leading dimension ld).
 * efie_bie2d_setup: pol 0 (TM, the paper's eq. 7 and 16) or 1 (TE, the other
 *   polarization, by the same Calderon structure: incident H_z, unknown the
 *   tangential current along z x n, N j = (j k/eta)(lambda, E_t), (G/2 - D) j =
 *   -(lambda, H_z), C_p = S_k~ G^-1 N_k + (G/2 + D_k~) G^-1 (G/2 - D_k) with
 *   D = D*^T, b_p = S_k~ G^-1 (j k/eta) e_t - (G/2 + D_k~) G^-1 h_z); assembles the
 *   four operators of C_p at k and k~ and the counterpart's first column (and its
 *   inverse's) from the spectra of its factors on the circle; the workspace must
 *   stay alive for the later calls.
 * efie_bie2d_apply: Y = op X for nvec rows, op 0: C_p, 1: C_p^T, 2: C_c, 3: C_c^-1,
 *   4: G^-1, 5: C_p - C_c.
 * efie_bie2d_rhs: e, h (and b_p if bp is not null) for plane waves of incidence
 *   angles phis (host, nrhs); TM: e = (lambda, E_z), h = (lambda, H_t); TE:
 *   e = (lambda, E_t), h = (lambda, H_z); synchronises.
 * efie_bie2d_skeleton: the range finder on A = C_p - C_p,c with the test matrix
 *   omega (dev, ncols x n rows, ncols >= block; the last block may be partial): *rank, the last projected block's
 *   largest column norm *est and the reference scale *ref (host); then
 *   V^T = U^H A, W = C_c^-1 U and the LU factors of I + V^T W.  Synchronises.
 *   EFIE_ERR_ARG if rank would exceed rmax or omega runs out; EFIE_ERR_BREAKDOWN
 *   if a factorization fails.
 * efie_bie2d_solve: X = C_p^-1 B by the Woodbury formula (nrhs rows, <= nvec).
 * efie_bie2d_factors: copies U (rank x n rows) and V^T (rank x n) into dev buffers.
 * efie_bie2d_counterpart: the first columns of C_p,c and of its inverse (dev, n).
 * efie_bie2d_farfield: 2-D far-field amplitude, phis dev (nphi), F dev (nrhs x
 *   nphi); pol 0 (TM): F[s][d] = int J_s exp(j k rhat_d . r) dS, echo width
 *   (k eta^2 / 4) |F|^2; pol 1 (TE): F[s][d] = int (rhat_d . n) J_s exp(j k rhat_d . r) dS,
 *   echo width (k / 4) |F|^2.
 * efie_bie2d_perimeter: the polygon perimeter of contour `which` (host).
 */
typedef struct efie_bie2d_s* efie_bie2d;
int efie_bie2d_create(const double* nodes, const double* circle_nodes, int64_t n, int q, efie_bie2d* out);
void efie_bie2d_destroy(efie_bie2d h);
int efie_bie2d_sizes(efie_bie2d h, int64_t rmax, int64_t block, int64_t nvec, size_t* table_bytes,
                     size_t* ws_bytes);
int efie_bie2d_upload(efie_bie2d h, void* dev, size_t bytes, hipStream_t stream);
int efie_bie2d_perimeter(efie_bie2d h, int which, double* perimeter);
int efie_bie2d_assemble(efie_bie2d h, int which, double k_re, double k_im, void* S, void* Dstar, void* Nm,
                        int64_t row0, int64_t nrows, int64_t col0, int64_t ncols, int64_t ld, hipStream_t stream);
int efie_bie2d_setup(efie_bie2d h, int pol, double k, double kt_re, double kt_im, int64_t rmax, int64_t block,
                     int64_t nvec, void* ws, size_t ws_bytes, hipStream_t stream);
int efie_bie2d_apply(efie_bie2d h, int op, const void* X, void* Y, int64_t nvec, hipStream_t stream);
int efie_bie2d_rhs(efie_bie2d h, const double* phis, int64_t nrhs, double eta, void* e, void* hv, void* bp,
                   hipStream_t stream);
int efie_bie2d_skeleton(efie_bie2d h, const void* omega, int64_t ncols, double tol, int64_t* rank, double* est,
                        double* ref, hipStream_t stream);
int efie_bie2d_solve(efie_bie2d h, const void* B, void* X, int64_t nrhs, hipStream_t stream);
int efie_bie2d_factors(efie_bie2d h, void* U, void* Vt, hipStream_t stream);
int efie_bie2d_counterpart(efie_bie2d h, void* col, void* col_inv, hipStream_t stream);
int efie_bie2d_farfield(efie_bie2d h, int pol, double k, const void* J, int64_t nrhs, const double* phis,
                        int64_t nphi, void* F, hipStream_t stream);

/* -------------------------------------------------------------- utilities */

/*
 * dst = src elementwise for count complex numbers, converting between complex128
 * and complex64 (round to nearest) when the dtypes differ.  Both dev.  Used to
 * store an operator or a preconditioner in complex64 for the mixed form.
 */
int efie_convert(const void* src, int src_dtype, void* dst, int dst_dtype, int64_t count, hipStream_t stream);

/* ------------------------------------------------------------ measurement */

/*
 * Optional HIP-event timing of the library's kernels (off by default).  While
 * enabled, every launch of the timed kernels is bracketed by two events on its
 * stream.  Kernel ids: 0 far-pair assembly, 1 near-pair assembly, 2 complex64
 * matrix-core GEMM, 3 GEMV, 4 FP64 GEMM, 5 Krylov vector kernels, 6 excitation,
 * 7 far field, 8 / 9 / 10 vertex gradient far pairs / near pairs / per-triangle
 * excitation and radiation terms, 11 the near pairs of the pair rows of the
 * Calderon build (beside its far pairs, on a second stream), 12 the mixed
 * solves' complex64 matrix-core products of at most 32 columns (the 32-row tile;
 * id 2 holds the others).  efie_prof_read waits for the recorded events and returns the
 * launch count, summed milliseconds and summed algorithmic work (real flops for
 * the GEMMs, 8 M n n per complex product; Z bytes read for the GEMVs; triangle
 * pairs for the gradient pair kernels and triangles for its per-triangle
 * kernel; 0 where not defined) since the last efie_prof_reset.  total_work may
 * be NULL.
 */
int efie_prof_enable(int on);
int efie_prof_reset(void);
int efie_prof_read(int kernel_id, int64_t* launches, double* total_ms, double* total_work);

#ifdef __cplusplus
}
#endif

#endif /* EFIE_H */
