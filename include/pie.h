/*
 * pie.h -- C ABI of the MI355X (gfx950) MLFMA library for the potential
 * integral equations (PIEs) of perfectly conducting surfaces,
 * after Gur & Ergul, "Solutions of New Potential Integral Equations Using
 * MLFMA Based on the Approximate Stable Diagonalization" (arXiv:1806.04164).
 *
 * Problem (Section 2, Eqs. (1)-(2)): a triangulated surface S in free space,
 * closed or open (Section 4 solves both a sphere and a flat patch), at
 * angular frequency w, exp(-i w t) convention; unknowns are the current J
 * expanded in RWG functions (one per interior edge, E of them; boundary
 * edges of an open surface carry none) and n.A expanded in pulse functions
 * (one per triangle, T of them), N = E + T.
 * Galerkin testing gives Z [a; b] = [b^J; b^A] with
 *   Z^JJ = mu0 <f_m, int f_n g>, Z^JA = <div f_m, int P_p g>,
 *   Z^AJ = <P_q, int div' f_n g>, Z^AA = w^2 eps0 <P_q, int P_p g>,
 *   g = exp(i k R)/(4 pi R); b^J = -<f_m, A^inc>, b^A = -i w eps0 <P_q, Phi^inc>.
 * The matrix-vector product is done with the MLFMA of Section 3: near-field
 * entries for one-box-buffer neighbours, and aggregation, diagonal
 * translation with the scaled plane waves of Eq. (4) and the modified
 * translation function of Eq. (5), and disaggregation for the rest.
 *
 * Conventions for every call:
 *  - Return value: PIE_OK (0), a negative error code, or a positive warning.
 *    No exception crosses the ABI.  pie_last_error() returns the message of
 *    the last failure on the calling thread.
 *  - Handles are opaque, owned by the library, released by *_destroy.
 *  - Arrays are owned by the caller.  "host" arrays are ordinary CPU memory;
 *    "device" arrays are device pointers on the operator's GPU.
 *  - Complex numbers are interleaved (re, im) doubles (complex128).
 *  - Multi-RHS vectors are [N][R], R contiguous, unknowns in canonical order:
 *    the E RWG coefficients in edge-table order, then the T pulse
 *    coefficients in triangle order.
 *  - Every argument is validated on the host before any device work, so
 *    argument errors are reported without a GPU.
 *  - An operator is used by one stream at a time; calls on the same operator
 *    from different streams without ordering race.
 */
#ifndef PIE_H
#define PIE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t pie_status;

#define PIE_OK 0
#define PIE_ERR_ARG (-1)         /* invalid argument (null, size, range)      */
#define PIE_ERR_MESH (-2)        /* non-manifold, degenerate or misoriented   */
#define PIE_ERR_NONFINITE (-3)   /* NaN or Inf in an input                    */
#define PIE_ERR_PRECISION (-4)   /* translation table out of range for the    */
                                 /* requested precision                      */
#define PIE_ERR_OOM (-5)         /* device or host allocation failed          */
#define PIE_ERR_HIP (-6)         /* HIP runtime error (message has details)   */
#define PIE_ERR_UNSUPPORTED (-7) /* option combination not implemented        */
#define PIE_WARN_NOT_CONVERGED 1 /* solver stopped at maxit above tolerance   */

#define PIE_FP32 32
#define PIE_FP64 64

typedef struct pie_mesh pie_mesh;
typedef struct pie_tree pie_tree;
typedef struct pie_op pie_op;

/* Copies the last error message of this thread into buf (NUL-terminated,
 * truncated to len) and returns the full message length. */
size_t pie_last_error(char* buf, size_t len);

/* Library version as major*10000 + minor*100 + patch. */
int32_t pie_version(void);

/* ------------------------------------------------------------------ mesh --
 * Section 2: RWG functions on the interior edges, pulses on the triangles.
 * V: host double [nv][3] vertex coordinates (metres).
 * T: host int32 [nt][3] vertex indices, counter-clockwise seen from outside.
 * Edges are the vertex pairs (a < b) in ascending order; T+ is the triangle
 * whose counter-clockwise cycle runs a->b.  Fails with PIE_ERR_MESH on a
 * degenerate triangle, an edge shared by more than two triangles or
 * inconsistent orientation; PIE_ERR_NONFINITE on NaN/Inf coordinates.
 * Boundary edges (open surfaces) carry no RWG function. */
pie_status pie_mesh_create(const double* V, int64_t nv, const int32_t* T,
                           int64_t nt, pie_mesh** out);
void pie_mesh_destroy(pie_mesh* m);
/* Section 4 (the sphere experiments): a closed sphere of the given radius
 * (metres) meshed as an icosphere with 20 * 4^subdiv triangles and
 * 10 * 4^subdiv + 2 vertices.  The 12 icosahedron vertices (0, a, b),
 * (a, b, 0), (b, 0, a) for a = -1, 1 and b = -g, g (g the golden ratio) are
 * put on the unit sphere; each subdivision splits every triangle into four
 * (v0 m01 m20, v1 m12 m01, v2 m20 m12, m01 m12 m20), a midpoint vertex
 * (0.5 (a + b) normalised) being appended when its edge is first met in
 * face order (edges v0v1, v1v2, v2v0); then vertices are scaled by radius.
 * jitter > 0 moves vertex v by jitter * h_v * (2u - 1) in each coordinate,
 * h_v its shortest edge, u the draw 3v + c (coordinate c) of SplitMix64
 * started at seed, top 53 bits scaled to [0, 1).  The arithmetic is
 * reproducible bit for bit (no contraction).  Then as pie_mesh_create.
 * PIE_ERR_ARG unless 0 <= subdiv <= 10, radius > 0, 0 <= jitter < 0.5. */
pie_status pie_mesh_icosphere(int32_t subdiv, double radius, double jitter,
                              uint64_t seed, pie_mesh** out);
/* Vertex and triangle counts, and (if non-NULL) host copies of the mesh's
 * double [nv][3] vertices and int32 [nt][3] triangles. */
pie_status pie_mesh_geometry(const pie_mesh* m, int64_t* nv, int64_t* nt,
                             double* V, int32_t* T);
/* nE: number of RWG functions, nT: number of triangles (pulses). */
pie_status pie_mesh_sizes(const pie_mesh* m, int64_t* nE, int64_t* nT);
/* Host int32 [nE][2] arrays (any may be NULL): edge vertices (a, b),
 * triangles (T+, T-), free vertices (p+, p-). */
pie_status pie_mesh_edges(const pie_mesh* m, int32_t* edges, int32_t* tri,
                          int32_t* free_vertex);

/* ------------------------------------------------------------------ tree --
 * Section 3: the object is enclosed in a cubic box (vertex bounding box,
 * side = its largest extent) divided recursively; level 1 is the root and
 * levels >= 3 are required (3 = single-level FMM).  Basis reference points:
 * RWG edge midpoint, pulse centroid.  Boxes of each level are the nonempty
 * ones in Morton order (bit b of x,y,z -> bits 3b,3b+1,3b+2).  Unknowns are
 * internally reordered by (finest box, RWG before pulse, canonical index).
 * Near field: finest boxes within one box in every direction.  Far field at
 * level l >= 3: same-level boxes not near but with near parents; offsets
 * (obs - src) are numbered 0..315 over [-3,3]^3 with max|.| >= 2 in
 * lexicographic (dx, dy, dz) order. */
pie_status pie_tree_build(const pie_mesh* m, int32_t levels, pie_tree** out);
void pie_tree_destroy(pie_tree* t);

#define PIE_TQ_NBOX 1      /* level: count = boxes                            */
#define PIE_TQ_COORDS 2    /* level: int64 [nb][3] integer box coordinates    */
#define PIE_TQ_PARENT 3    /* level >= 2: int64 [nb] parent index             */
#define PIE_TQ_PERM 4      /* int64 [N] canonical unknown at box-order slot   */
#define PIE_TQ_BOXPTR 5    /* int64 [nb_L+1] box-order ranges of finest boxes */
#define PIE_TQ_NEAR_PTR 6  /* int64 [nb_L+1] CSR of near boxes (incl. self)   */
#define PIE_TQ_NEAR_IDX 7  /* int64 [nnz]                                     */
#define PIE_TQ_IL_PTR 8    /* level >= 3: int64 [nb+1] interaction-list CSR   */
#define PIE_TQ_IL_SRC 9    /* level >= 3: int64 [nnz] source boxes            */
#define PIE_TQ_IL_OFF 10   /* level >= 3: int64 [nnz] offset ids 0..315       */
/* Two-call query: with data == NULL only *count is set; otherwise data (host,
 * int64, at least *count entries as returned by the first call) is filled. */
pie_status pie_tree_query(const pie_tree* t, int32_t what, int32_t level,
                          int64_t* count, int64_t* data);

/* -------------------------------------------------------------- operator --
 * MLFMA parameters (Eqs. (4)-(5)).  The paper tabulates the truncation
 * number tau and scale factor s per box size in a reference that is not
 * reproduced; here s_l = min(1, k d_l / x) per level, so that the scaled box
 * size k d_l / s_l equals x wherever s < 1, and (tau, x) default per far
 * precision to values chosen by measured error against the dense matrix
 * (sampled rows, 4 to 8 levels) and by the rounding that the sampled
 * translation amplifies by about (2 tau + 1)!!/(2 x)^tau:
 *   far FP64: x = 0.08 for trees of up to 5 levels, 0.07 for 6 and 0.06
 *             for 7 or more (deeper trees accumulate more of the inter-level
 *             rescaling error, which grows as x^2); the truncation number
 *             per level from its box size: tau_l = 7 for k d_l <= 0.8, 8 for
 *             <= 1.6, 9 for <= 3.2, 10 for <= 4.8 (Section 3: as boxes grow, s -> 1 and
 *             Eq. (5) becomes the ordinary translation function, which
 *             needs more terms; measured against sampled dense rows at 1 to
 *             3 wavelengths); PIE_ERR_UNSUPPORTED for larger level-3 boxes;
 *   far FP32: tau = 4, x = 0.15, k d_3 <= 1.
 * A caller's tau (> 0) applies at every level and covers k d_l up to 1.0
 * (tau < 7), 1.6 (7, 8), 3.2 (9) or 4.8 (>= 10).  Every level uses the
 * k-space samples of the largest tau_l (so no interpolation between
 * levels); the inter-level filter keeps degrees up to the parent level's
 * tau_l.
 * Near/far split (Section 3 does not state it): Z^JA = G S, Z^AJ = S G^T and
 * Z^AA = w^2 eps0 S share the scalar operator S_qp = <P_q, int P_p g> (G: the
 * RWG divergence per triangle).  S is applied per triangle -- each triangle's
 * sources sigma = x_A and u = div J + w^2 eps0 x_A radiate and are received at
 * the finest box of its centroid, and a triangle pair is near when those
 * boxes are -- and the vector part mu0 <f_m, int f_n g> per RWG function (the
 * box of its edge midpoint), so the approximation keeps that identity:
 * divergence-free currents have no scalar source and the JA block keeps the
 * charge null vector of the dense matrix, which keeps low-frequency solves
 * as accurate as the operator.
 * k-space samples: n_theta Gauss-Legendre points in cos(theta) (default
 * tau+1, tau the largest tau_l) times n_phi uniform phi (default 2 tau + 2).
 * near_prec: storage and arithmetic of the near-field SpMM.
 * far_prec: patterns, translation and shifts.
 * Tables (translation, filters) are always computed in FP64. */
typedef struct pie_options {
  int32_t version;   /* must be 1                                      */
  int32_t near_prec; /* PIE_FP32 or PIE_FP64                           */
  int32_t far_prec;  /* PIE_FP32 or PIE_FP64                           */
  int32_t tau;       /* 0: default for far_prec (per level, above)     */
  double x;          /* 0: default for far_prec                        */
  int32_t n_theta;   /* 0: tau + 1                                     */
  int32_t n_phi;     /* 0: 2 tau + 2                                   */
  int32_t max_rhs;   /* calls take up to this many RHS (>= 1); the far-
                        field workspace holds min(max_rhs, 64) columns,
                        wider calls run in passes of 64 */
  int32_t flags;     /* 0, or PIE_OPT_* bits below (the former reserved
                        field; version 1 callers pass 0)              */
} pie_options;

/* pie_options.flags: run the FP64 inter-level shifts on the matrix cores at
 * every level.  By default they run there only where a level has enough
 * (parent group, 32-sample block) work items to fill the device; this
 * option exists so that small trees can pin those kernels against the
 * oracle.  The result differs from the default only by FP64 rounding. */
#define PIE_OPT_MATRIX_SHIFTS 1

/* Fills *o with defaults (FP64 near and far, max_rhs 1). */
void pie_options_default(pie_options* o);

/* Builds the operator on the current HIP device: device geometry, near-field
 * fill (FP64 arithmetic, closed-form singular parts for triangle pairs that
 * share a vertex, symmetrised), translation tables and inter-level filters.
 * mesh and tree must stay alive until the operator is destroyed.
 * stream: hipStream_t (NULL = default stream); the call returns after the
 * setup work on it has completed. */
pie_status pie_operator_create(const pie_mesh* m, const pie_tree* t,
                               double freq_hz, const pie_options* opt,
                               void* stream, pie_op** out);
void pie_operator_destroy(pie_op* op);

#define PIE_OI_N 1          /* number of unknowns                         */
#define PIE_OI_Q 2          /* k-space samples per level                  */
#define PIE_OI_TAU 3        /* largest truncation number over the levels  */
#define PIE_OI_NEAR_BLOCKS 4 /* stored (upper-triangle) near blocks       */
#define PIE_OI_NEAR_ENTRIES 5 /* stored near-field entries                */
#define PIE_OI_NEAR_BYTES 6  /* bytes of stored near-field entries        */
#define PIE_OI_NBOX_FINEST 7
#define PIE_OI_IL_PAIRS 8    /* interaction-list pairs over all levels    */
#define PIE_OI_INCIDENCES 9  /* (finest box, triangle) incidences         */
#define PIE_OI_DEVICE_BYTES 10 /* device memory held by the operator      */
#define PIE_OI_NEAR_ENTRIES_RWG 11 /* stored RWG-RWG near entries          */
#define PIE_OI_NEAR_ENTRIES_TRI 12 /* stored triangle-triangle entries of  */
                                   /* the scalar operator (applied to x_A  */
                                   /* and u)                               */
/* truncation number of Eq. (5) at level l (3..L) */
#define PIE_OI_TAU_LEVEL(l) (100 + (l))
pie_status pie_operator_info(const pie_op* op, int32_t what, int64_t* value);
/* Scale factor s and kappa = k/s at level l (3..L). */
pie_status pie_operator_level(const pie_op* op, int32_t level, double* s,
                              double* kappa, double* box_side);

/* ------------------------------------------------------------------ MVM --
 * y = Z x (adjoint = 0) or y = Z^H x (adjoint = 1) for R right-hand sides,
 * 1 <= R <= max_rhs.  x, y: device complex128 [N][R], canonical order, must
 * not overlap.  Asynchronous on stream (hipStream_t, NULL = default).
 * Z^H x = conj(Z conj(x)) because the Galerkin matrix and its MLFMA
 * approximation are complex symmetric (Z = Z^T); the adjoint path folds the
 * two conjugations into its input and output kernels.
 * Columns are processed in passes of at most min(max_rhs, 64).  Passes of 16
 * or more columns run batched kernels (matrix-core near field, aggregation,
 * shifts and reception; grouped row translation), narrower passes the
 * single-column kernels.  A column's result is bitwise the same for every
 * pass width on the same side of that boundary; across it the summation
 * order differs (FP64 rounding, amplified by the sampled translation). */
pie_status pie_matvec(pie_op* op, const void* x, void* y, int64_t R,
                      int32_t adjoint, void* stream);

/* Near-field part only (y = Z_near x) and far-field part only (y = Z_far x),
 * same conventions as pie_matvec (used for per-stage parity and timing). */
pie_status pie_matvec_near(pie_op* op, const void* x, void* y, int64_t R,
                           void* stream);
pie_status pie_matvec_far(pie_op* op, const void* x, void* y, int64_t R,
                          void* stream);

/* ------------------------------------------------------------ profile --
 * Stage timing with HIP events recorded on the MVM stream around every
 * kernel launch (each stage's events bracket exactly its kernels).
 * pie_profile_enable(op, 1) clears the counters and starts recording;
 * pie_profile_read waits for the recorded events and returns, per stage,
 * the summed milliseconds (host double [PIE_NSTAGES]) and the number of
 * launches (host int64 [PIE_NSTAGES]); either may be NULL. */
#define PIE_STAGE_PERMUTE 0   /* canonical x -> box order (near precision) */
#define PIE_STAGE_NEAR 1      /* near-field SpMM                           */
#define PIE_STAGE_AGGREGATE 2 /* finest-level radiation patterns           */
#define PIE_STAGE_SHIFT_UP 3  /* child -> parent shifts                    */
#define PIE_STAGE_TRANSLATE 4 /* interaction-list translations              */
#define PIE_STAGE_RECEIVE 5   /* reception + near join + output permutation */
#define PIE_STAGE_SHIFT_DOWN 6 /* parent -> child shifts                   */
#define PIE_NSTAGES 7
pie_status pie_profile_enable(pie_op* op, int32_t on);
pie_status pie_profile_read(pie_op* op, double* ms, int64_t* launches);

/* ----------------------------------------------------------- schedule --
 * Placement of the MVM's kernels on streams.  Every schedule computes the
 * same result bit for bit: neither the arithmetic nor its order depends on
 * it, only the overlap of independent stages.
 *   near_fork: PIE_NEAR_SERIAL runs the near field, then the far chain, on
 *     the caller's stream; PIE_NEAR_FORK_START runs the near field on a
 *     second stream from the start; PIE_NEAR_FORK_AFTER_AGGREGATE forks it
 *     after the finest-level aggregation.  The reception joins it.
 *   il_fork: 0 keeps the finest level's interaction-list translation on
 *     the caller's stream; 1 runs it on a third stream forked after the
 *     aggregation (concurrent with the upward shifts); 2 forks it after
 *     the first upward shift (concurrent with the coarse levels); 3 runs
 *     the translation of every level >= 4 on a stream of its own, forked
 *     as soon as that level's patterns exist; 4 runs the translations of
 *     all levels in one launch after the upward pass (no stream fork).
 *   max_chunk: widest register group of RHS columns inside a kernel (1, 2
 *     or 4; the operator's own limit from its LDS budget applies).
 * Default: PIE_NEAR_FORK_START, il_fork 1, max_chunk 4. */
#define PIE_NEAR_SERIAL 0
#define PIE_NEAR_FORK_START 1
#define PIE_NEAR_FORK_AFTER_AGGREGATE 2
typedef struct pie_schedule {
  int32_t version; /* must be 1 */
  int32_t near_fork;
  int32_t il_fork;
  int32_t max_chunk;
} pie_schedule;
pie_status pie_schedule_get(const pie_op* op, pie_schedule* out);
/* PIE_ERR_ARG for an unknown near_fork, il_fork not 0..4, or max_chunk not
 * 1, 2 or 4. */
pie_status pie_schedule_set(pie_op* op, const pie_schedule* sch);

/* Autotuner: times every distinct schedule on R right-hand sides in two
 * rounds (each round one warm-up, then reps MVMs per schedule, HIP events
 * on stream; a schedule's time is its faster round), keeps the fastest
 * on the operator and returns it in *chosen and its time per MVM in *ms
 * (either may be NULL).  x, y: caller-owned device complex128 [N][R] work
 * vectors (x is read, y overwritten).  Stage profiling must be off.
 * Synchronizes the stream. */
pie_status pie_autotune(pie_op* op, const void* x, void* y, int64_t R,
                        int32_t reps, void* stream, pie_schedule* chosen,
                        double* ms);

/* ------------------------------------------------------------- graphs --
 * A captured MVM: the kernels of y = Z x (adjoint = 0) or Z^H x for fixed
 * x, y and R, with the operator's schedule at capture time, recorded once
 * into a HIP graph (captured on a private stream; the operator's side
 * streams join it through events) and replayed with one launch.  A replay
 * uses the operator's workspace: replays and other calls on the same
 * operator must not overlap.  Stage profiling must be off when capturing.
 * The graph must be destroyed before its operator. */
typedef struct pie_graph pie_graph;
pie_status pie_graph_create(pie_op* op, const void* x, void* y, int64_t R,
                            int32_t adjoint, pie_graph** out);
pie_status pie_graph_launch(pie_graph* g, void* stream);
/* Uneven batch: one graph holding the MVMs of nobj distinct operators
 * (objects of different sizes and frequencies, each with its own device x,
 * y [N_i][R_i] and R_i), captured one after another (each with its own
 * stream forks), so that one launch runs every object.  Each object's
 * result equals its own pie_matvec bit for bit.  PIE_ERR_ARG for a
 * repeated operator or an invalid per-object call. */
pie_status pie_graph_create_batch(pie_op* const* ops, int32_t nobj,
                                  const void* const* xs, void* const* ys,
                                  const int64_t* Rs, int32_t adjoint,
                                  pie_graph** out);
void pie_graph_destroy(pie_graph* g);

/* --------------------------------------------------------- uneven batch --
 * Uneven batch (the sphere sweep of Section 4 as one workload: objects of
 * different sizes, frequencies, precisions and RHS counts): the MVMs
 * y_i = Z_i x_i (or the adjoint products) of several distinct operators in
 * one call.  pie_batch_create keeps one stream and event per object
 * (default priority); pie_batch_matvec forks them from `stream`, runs object
 * i's MVM on its own stream (its schedule's side streams as in pie_matvec)
 * so that the objects' kernels run concurrently, and joins them back into
 * `stream` before returning (asynchronous with respect to the host).  xs[i],
 * ys[i]: device complex128 [N_i][Rs[i]], as for pie_matvec; each result
 * equals that object's own pie_matvec bit for bit.  PIE_ERR_ARG on null
 * arguments, an operator given twice, a bad R or stage profiling on.  The
 * batch holds the operator handles, not ownership; destroy it before them.
 * Calls on one batch must not overlap. */
typedef struct pie_batch pie_batch;
pie_status pie_batch_create(pie_op* const* ops, int32_t nobj, pie_batch** out);
pie_status pie_batch_matvec(pie_batch* b, const void* const* xs,
                            void* const* ys, const int64_t* Rs,
                            int32_t adjoint, void* stream);
void pie_batch_destroy(pie_batch* b);

/* ---------------------------------------------------------------- RHS --
 * Plane waves E^inc = amp_r pol_r exp(i k khat_r . r) (E0 = 1 V/m scale).
 * khat, pol: host double [R][3] (unit, orthogonal); amp: host complex128 [R].
 * gauge 0 (Lorenz, finite at zero frequency):
 *   Phi = -amp (pol.r) e^{ik khat.r}, A = -(amp/c0)(pol.r) khat e^{ik khat.r};
 * gauge 1: Phi = 0, A = E^inc/(i w).
 * b: device complex128 [N][R]:  b^J_m = -<f_m, A^inc>,
 * b^A_q = -i w eps0 <P_q, Phi^inc>, with the 7-point rule. */
pie_status pie_rhs_planewave(pie_op* op, int64_t R, const double* khat,
                             const double* pol, const double* amp,
                             int32_t gauge, void* b, void* stream);

/* -------------------------------------------------------------- solve --
 * GMRES(restart) for Z x = b (Section 4) on the symmetrically equilibrated
 * system D Z D (D = diag |Z_ii|^-1/2), FP64 orthogonalisation and residual.
 * Each outer refinement step solves the correction equation with the
 * operator's own precision and recomputes the residual b - Z x with the
 * residual operator (if res_op is NULL, op itself).  x: device complex128
 * [N][R] (input: initial guess if use_x0, output: solution).
 * Residuals are relative and measured in the equilibrated norm,
 * ||D (b - Z x)|| / ||D b||, the norm GMRES minimises (the rows of Eqs. (1)
 * and (2) carry different units; at low frequency their scales differ by
 * orders of magnitude, so the plain 2-norm weighs one block only).
 * info (host, may be NULL) receives iterations and final relative residual
 * per RHS. Returns PIE_WARN_NOT_CONVERGED if any RHS missed tol. */
typedef struct pie_solve_opts {
  int32_t version;    /* 2 (1: the fields up to adjoint, precond = 0)  */
  int32_t restart;    /* Krylov dimension per cycle (default 100)     */
  int32_t maxit;      /* total inner iterations per RHS (default 1000) */
  int32_t refine;     /* outer refinement steps (default 1 = none)    */
  double tol;         /* relative residual target (default 1e-6)      */
  double inner_tol;   /* inner tolerance per refinement (default tol) */
  int32_t use_x0;     /* 1: x holds the initial guess                 */
  int32_t adjoint;    /* 1: solve Z^H x = b                           */
  int32_t precond;    /* 1: right block-diagonal preconditioner: the   */
                      /* inverses of the finest boxes' FP64 self      */
                      /* blocks (built on the first such solve and    */
                      /* kept with the operator: 16 sum n_b^2 bytes   */
                      /* of device memory; the inversion runs on the  */
                      /* host, O(sum n_b^3), up to 16 threads).       */
                      /* Suited to open surfaces; on closed surfaces  */
                      /* a box's local charge modes make M^-1 huge    */
                      /* and it slows or stalls GMRES                 */
} pie_solve_opts;
typedef struct pie_solve_info {
  int32_t iterations; /* total inner iterations (max over RHS)        */
  int32_t refinements;
  double rel_residual; /* max over RHS, with the residual operator     */
} pie_solve_info;
void pie_solve_opts_default(pie_solve_opts* o);
pie_status pie_solve(pie_op* op, pie_op* res_op, const void* b, void* x,
                     int64_t R, const pie_solve_opts* opts,
                     pie_solve_info* info, void* stream);

/* For callers that cannot allocate device memory (serving loops that must
 * not call hipMalloc, harnesses that forbid it): pie_solve with the same
 * arguments, results and status codes, but the solver's device workspace is
 * a fixed array that the library holds on each GPU from the first call
 * until the process ends (PIE_SOLVE_NOALLOC_BYTES = 128 MiB per GPU), so the
 * call allocates nothing.  It needs 16 N R (restart + 7) + 16 R (restart + 2)
 * bytes and returns PIE_ERR_ARG, before any device work, when that exceeds
 * the array (e.g. N = 51 200, R = 1 allows restart <= 156).  precond = 1
 * requires the preconditioner to exist already (pie_precond_apply or a
 * pie_solve with precond = 1 builds it; building allocates), else
 * PIE_ERR_ARG.  Every call on a GPU shares that GPU's array: calls that
 * overlap on one GPU (from different threads or streams) race and must be
 * serialised by the caller.  The operators' own workspaces are allocated at
 * pie_operator_create, so the MVMs inside allocate nothing either. */
#define PIE_SOLVE_NOALLOC_BYTES (128u << 20)
pie_status pie_solve_noalloc(pie_op* op, pie_op* res_op, const void* b,
                             void* x, int64_t R, const pie_solve_opts* opts,
                             pie_solve_info* info, void* stream);

/* Block-diagonal preconditioner of the solve (precond = 1): y = M^-1 x with
 * M = blockdiag(Z_bb) over the finest boxes b (FP64 self blocks, inverted on
 * the host at the first use and kept with the operator), for callers with
 * their own Krylov solver.  x, y: device complex128 [N][R], canonical order,
 * not overlapping. */
pie_status pie_precond_apply(pie_op* op, const void* x, void* y, int64_t R,
                             void* stream);

/* ------------------------------------------------------- near-zone charge --
 * Section 2 (the paragraph after Eq. (2)): the surface charge density for
 * near-zone fields, rho = i w eps0 n.A - eps0 n.grad(Phi), where
 * sigma = n.grad(Phi) solves Eq. (3),  int_S sigma(r') g(r,r') dr' = Phi^inc(r)
 * on S.  sigma is expanded in the pulse functions and Eq. (3) is tested with
 * them: S sigma = phi, S_qp = <P_q, int P_p g> (the pulse-pulse block of Z
 * divided by w^2 eps0, applied with the same MLFMA), phi_q = <P_q, Phi^inc>
 * for R plane waves (khat, pol, amp and gauge as in pie_rhs_planewave; use the
 * gauge of the PIE right-hand side).  GMRES on the equilibrated pulse block
 * with opts->tol, restart, maxit, refine, inner_tol (opts NULL: defaults;
 * adjoint must be 0).
 * x:     device complex128 [N][R], the PIE solution (its pulse rows are n.A);
 *        may be NULL when rho is NULL.
 * sigma: device complex128 [T][R] out, n.grad(Phi) per triangle (triangle order).
 * rho:   device complex128 [T][R] out (C/m^2 for E0 = 1 V/m), or NULL.
 * Allocates a 2 N R complex128 workspace.  Returns PIE_WARN_NOT_CONVERGED if
 * GMRES stops above tol (the outputs hold the last iterate). */
pie_status pie_charge(pie_op* op, int64_t R, const double* khat,
                      const double* pol, const double* amp, int32_t gauge,
                      const void* x, void* sigma, void* rho,
                      const pie_solve_opts* opts, pie_solve_info* info,
                      void* stream);

/* ---------------------------------------------------------- far field --
 * F(rhat) = lim r e^{-ikr} E^s = (i w mu0 / 4 pi)(I - rhat rhat).
 *           int J(r') exp(-i k rhat.r') dr',  J = sum a_n f_n.
 * x: device complex128 [N][R]; dirs: host double [nd][3] unit vectors;
 * F: device complex128 [R][nd][3]. */
pie_status pie_farfield(pie_op* op, const void* x, int64_t R,
                        const double* dirs, int64_t nd, void* F,
                        void* stream);

/* Adjoint of pie_farfield (for gradients of far-field quantities):
 * gx = Phi^H gF with F = Phi x as defined above.  gF: device complex128
 * [R][nd][3]; gx: device complex128 [N][R] (pulse rows set to zero). */
pie_status pie_farfield_adjoint(pie_op* op, const void* gF, int64_t R,
                                const double* dirs, int64_t nd, void* gx,
                                void* stream);

#ifdef __cplusplus
}
#endif
#endif /* PIE_H */
