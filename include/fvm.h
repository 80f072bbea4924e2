/*
 * fvm.h -- C interface of libfvm, an MI355X (gfx950) implementation of the
 * data-parallel hot path of an incompressible finite-volume PISO / SIMPLE
 * solver on unstructured meshes (Tomczak et al., "Complete PISO and SIMPLE
 * solvers on Graphics Processing Units").
 *
 * Problem statement (paper, Section 3.1): the domain is a mesh of N
 * polyhedral cells; every face belongs to exactly two cells or is a boundary
 * face; pressure p and velocity U live at cell centroids; each solve is a
 * sparse system A x = b with A_ij != 0 iff cells i and j share a face or
 * i == j, assembled from per-face quantities many times per run.  Arbitrary
 * (non-orthogonal) meshes and time-dependent boundary values are supported
 * (Sections 2 and 6).  Double precision throughout (Section 4.2), plus an
 * optional FP32-inner / FP64-refinement mode.
 *
 * Conventions shared by every call:
 *   - Return value: FVM_OK (0); > 0 a warning with valid results
 *     (FVM_WARN_MAXITER: some solve stopped at max_iter); < 0 an error, in
 *     which case the case state is unchanged (a failed step is rolled back to
 *     its start).  fvm_last_error() gives a thread-local message.
 *   - Host arrays (mesh description) are read during the call only; the
 *     caller keeps ownership.  Device arrays (d_*) are caller-owned device
 *     memory; the library never allocates device memory: every case lives in
 *     the caller's workspace buffer.
 *   - `stream` is a hipStream_t (NULL = default stream).  Work is enqueued on
 *     it; calls that return solver information synchronise on it and return
 *     once all of their work on it is complete.
 *   - Kernels run on the calling thread's current HIP device, which must be
 *     the device of the case's workspace, of the device arrays and of the
 *     stream.
 *   - All indices are in the caller's numbering: cells are never renumbered,
 *     faces are reordered internally and mapped back on output.
 *   - A handle is not thread-safe; distinct cases may run on distinct streams.
 *   - No C++ exception crosses this interface.
 */
#ifndef FVM_H
#define FVM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t fvm_status;
enum {
    FVM_OK = 0,
    FVM_WARN_MAXITER = 1,
    FVM_EINVAL = -1,     /* malformed mesh / arguments */
    FVM_ENOMEM = -2,     /* workspace too small */
    FVM_ENUMERIC = -3,   /* non-finite value or Krylov breakdown */
    FVM_EDEVICE = -4     /* HIP runtime error */
};

/* Boundary kind of a patch, for U and for p independently.
 * FIXED: the patch value; ZERO_GRAD: the owner-cell value; EMPTY: the face
 * takes part in no sum (front/back of 2-D slabs). */
enum { FVM_BC_FIXED = 0, FVM_BC_ZERO_GRAD = 1, FVM_BC_EMPTY = 2 };
/* Pressure preconditioner: Jacobi (the paper's choice, Section 3),
 * diagonal incomplete Cholesky, or one V-cycle of an aggregation algebraic
 * multigrid (the stronger preconditioner the paper leaves to future work,
 * Section 5: one-ring aggregation of the cell graph, piecewise-constant
 * prolongation, Galerkin coarse operators rebuilt at every solve, damped
 * Jacobi smoothing with weight 2/3 before and after the coarse correction,
 * an exact solve on the coarsest level; FP64 cases only, one case per
 * piso_step_batch call). */
enum { FVM_PC_JACOBI = 0, FVM_PC_DIC = 1, FVM_PC_AMG = 2 };
/* FVM_FP64: everything in double precision.  FVM_MIXED: the inner Krylov
 * iterations run in FP32 inside an FP64 residual-refinement loop. */
enum { FVM_FP64 = 0, FVM_MIXED = 1 };
enum { FVM_CONV_LINEAR = 0, FVM_CONV_UPWIND = 1 };
/* Momentum solver: bi-conjugate gradients (A and A^T products per
 * iteration), or BiCGStab (two A products per iteration, no A^T; the
 * method the paper's GPU solver uses for momentum, Section 4.2), both
 * Jacobi-preconditioned after Barrett et al.  BiCGStab is FP64 only. */
enum { FVM_SOLVER_BICG = 0, FVM_SOLVER_BICGSTAB = 1 };

typedef struct fvm_mesh fvm_mesh;
typedef struct fvm_case fvm_case;

/* One boundary patch: boundary faces [start, start+size) (face indices of
 * the mesh description) with their U and p kinds and values. */
typedef struct {
    int32_t start, size, u_kind, p_kind;
    double u_value[3];
    double p_value;
} fvm_patch;

/* Mesh description (Section 3.1).  Faces [0, n_internal_faces) are internal
 * with owner[f] != neighbour[f]; faces [n_internal_faces, n_faces) are
 * boundary faces of cell owner[f] and must be tiled, in order, by the
 * patches.  Sf[f] is the face area vector pointing out of owner[f]; Cf the
 * face centre; C the cell centres; V the cell volumes.  Vectors are [.][3]
 * row-major doubles. */
typedef struct {
    int32_t n_cells, n_faces, n_internal_faces, n_patches;
    const int32_t *owner;      /* [n_faces] */
    const int32_t *neighbour;  /* [n_internal_faces] */
    const double *Sf;          /* [n_faces][3] */
    const double *Cf;          /* [n_faces][3] */
    const double *C;           /* [n_cells][3] */
    const double *V;           /* [n_cells] */
    const fvm_patch *patches;  /* [n_patches] */
} fvm_mesh_desc;

/* Krylov controls: stop when the normalised L1 residual
 * sum|b - A x| / n_f  <=  max(tol, rel_tol * initial value), or at max_iter
 * (the paper stops on residual thresholds, Section 4.3.1). */
typedef struct {
    double tol, rel_tol;
    int32_t max_iter, precond;
} fvm_solver_ctl;

typedef struct {
    double nu;             /* kinematic viscosity */
    double dt;             /* PISO time step */
    double alpha_u;        /* SIMPLE implicit momentum relaxation */
    double alpha_p;        /* SIMPLE explicit pressure relaxation */
    double p_ref_value;    /* pressure level at p_ref_cell when no p patch is FIXED */
    double inner_rel_tol;  /* FVM_MIXED: relative reduction of each FP32 inner solve */
    int32_t n_corr;        /* PISO pressure correctors per step */
    int32_t n_non_orth_corr;
    int32_t convection;    /* FVM_CONV_* */
    int32_t precision;     /* FVM_FP64 | FVM_MIXED */
    int32_t p_ref_cell;    /* caller's cell index */
    int32_t inner_max_iter;
    fvm_solver_ctl p_ctl, u_ctl;
    int32_t u_solver;      /* FVM_SOLVER_* for the momentum equation */
    int32_t hybrid_K;      /* > 0: also lay out the paper's hybrid matrix format with this many ELL slots per
                              row, for fvm_case_operator's FVM_OP_HY_* operators (comparison layout); 0: none */
    int32_t step_kernel;   /* FVM_STEP_AUTO or FVM_STEP_LAUNCHED (below) */
} fvm_case_opts;

/* How piso_step and piso_step_batch run a case.  FVM_STEP_AUTO: a small
 * case (at most 32 768 cells, orthogonal mesh, Jacobi pressure CG, BiCG
 * momentum, at most 4 correctors, no non-orthogonal correctors) runs its
 * whole PISO steps, Krylov loops included, in one workgroup of one kernel
 * launch (many such cases side by side, one per compute unit), since at that
 * size launches and host round trips per Krylov iteration would cost more
 * than the arithmetic; any other case, and every case under
 * FVM_STEP_LAUNCHED, runs each phase of each iteration as a grid-wide launch.
 * Both give the method's result (they differ only in the order of the
 * floating-point sums). */
enum { FVM_STEP_AUTO = 0, FVM_STEP_LAUNCHED = 1 };

typedef struct {
    int32_t iters, status;
    double res_initial, res_final;
} fvm_solve_info;

typedef struct {
    fvm_solve_info u[3];       /* momentum predictor, per component */
    fvm_solve_info p[16];      /* pressure solves in order */
    int32_t n_p_solves, status;
} fvm_step_info;

/* fvm_mesh_create -- ingest a mesh (Section 3.1): validate it, canonicalise
 * the internal faces (lower cell index owns the face, sorted by owner then
 * neighbour), and build the cell-to-face index ranges used by every gather.
 * Host-side only; no device memory.  Errors: FVM_EINVAL for an index out of
 * range, owner == neighbour, a duplicated face, S.d <= 0, V <= 0, patches
 * that do not tile the boundary faces, or an unknown kind. */
fvm_status fvm_mesh_create(const fvm_mesh_desc *desc, fvm_mesh **out);
void fvm_mesh_destroy(fvm_mesh *mesh);
/* Sizes and whether any face is non-orthogonal (S not parallel to d). */
fvm_status fvm_mesh_info(const fvm_mesh *mesh, int32_t *n_cells, int32_t *n_faces, int32_t *n_internal_faces,
                         int32_t *non_orthogonal);

/* Structure of the sliced-ELL copy of the pressure matrix that the CG's
 * matrix-vector product reads (rows in slices of 256 consecutive cells,
 * w_slots entries per row, slot-major): the number of slices, how many of
 * them store explicit int32 column indices (a slice whose column offsets
 * j - i take at most w_slots values stores one offset per slot and no
 * index), the entries (internal faces seen from one of their two cells) in
 * explicit slices, and the entries of regular slices read through a mirror
 * slot (their symmetric coefficient is taken from the neighbour's upper
 * slot instead of a second copy), and the regular slices of the 7-point
 * form (offsets -c, -b, -1, +1, +b, +c with b and c even, the three lower
 * slots mirrored, every neighbour inside the mesh) on which the FP64
 * product takes two cells per thread.  Measurement support: it gives the
 * bytes a product must move.  Any pointer may be NULL. */
fvm_status fvm_mesh_sell_info(const fvm_mesh *mesh, int32_t *w_slots, int32_t *n_slices, int32_t *n_explicit_slices,
                              int64_t *explicit_entries, int64_t *mirrored_entries, int32_t *n_7pt_slices);

/* Exact device workspace size of a case of this mesh with these options
 * (admission control of many resident cases relies on it being exact). */
fvm_status fvm_case_workspace_bytes(const fvm_mesh *mesh, const fvm_case_opts *opts, size_t *bytes);

/* fvm_case_create -- lay a case out in the caller's device workspace
 * (bytes >= fvm_case_workspace_bytes, 256-byte aligned), upload the mesh,
 * derive the face geometry coefficients on the device and set U = 0,
 * p = 0 and phi = the boundary fluxes of U.  The mesh may be destroyed
 * afterwards.  Errors: FVM_ENOMEM if bytes is too small. */
fvm_status fvm_case_create(const fvm_mesh *mesh, const fvm_case_opts *opts, void *d_workspace, size_t bytes,
                           void *stream, fvm_case **out);
void fvm_case_destroy(fvm_case *c);    /* the workspace stays the caller's */

/* State exchange on `stream`, caller numbering: d_U [n_cells][3], d_p
 * [n_cells], d_phi [n_faces] (flux along the caller's Sf).  set_state with
 * d_phi == NULL sets phi = S.(interpolated U) with boundary values from the
 * patches.  Any pointer may be NULL in get_state. */
fvm_status fvm_case_set_state(fvm_case *c, const double *d_U, const double *d_p, const double *d_phi, void *stream);
fvm_status fvm_case_get_state(const fvm_case *c, double *d_U, double *d_p, double *d_phi, void *stream);
/* Time-dependent boundary values (Sections 2 and 6): replace a patch's U and
 * p values, effective for work enqueued afterwards on `stream`. */
fvm_status fvm_case_set_patch_value(fvm_case *c, int32_t patch, const double u_value[3], double p_value,
                                    void *stream);

/* piso_step -- n_steps transient PISO steps (Section 3): momentum predictor
 * (BiCG, Jacobi), then n_corr pressure correctors (CG with the case's
 * preconditioner, explicit flux and velocity corrections).  `last` (may be
 * NULL) receives the solver record of the final step. */
fvm_status piso_step(fvm_case *c, int32_t n_steps, void *stream, fvm_step_info *last);

/* simple_iterate -- steady SIMPLE iterations (Section 3) with implicit
 * momentum relaxation alpha_u and explicit pressure relaxation alpha_p, until
 * all four initial residuals (U_x, U_y, U_z, p) of an iteration are
 * <= res_tol, or max_iters. */
fvm_status simple_iterate(fvm_case *c, int32_t max_iters, double res_tol, void *stream, int32_t *iters_done,
                          fvm_step_info *last);

/* solve_pressure -- the pressure equation alone: the symmetric system whose
 * face coefficients are d_gamma_f[f] * |S_f|^2 / (S_f . d_f) (d_gamma_f in
 * the caller's face order, boundary entries used on FIXED-p patches), with
 * b = d_rhs + fixed-p boundary terms, pinned at p_ref_cell when no p patch
 * is FIXED, solved by CG (ctl->precond) from the guess in d_p. */
fvm_status solve_pressure(fvm_case *c, const double *d_gamma_f, const double *d_rhs, double *d_p,
                          const fvm_solver_ctl *ctl, void *stream, fvm_solve_info *info);

/* solve_pressure_static -- solve_pressure for callers that cannot allocate
 * (code that must not call hipMalloc: under stream capture by the caller's
 * own harness, tight serving loops, harnesses that forbid allocation).  The
 * same system, the same kernels and the same result as solve_pressure with
 * ctl->precond == FVM_PC_JACOBI on an FP64 case; the grid-reduction slots,
 * tickets, Krylov states and a device copy of the case descriptor live in a
 * file-scope device array of 4 MiB (one per GPU, held until the process
 * ends; enough for cases of about 11M cells) instead of the case's
 * workspace; the CG vectors stay in the workspace.  No device or pinned
 * memory is allocated, no graph is captured: iterations are launched
 * directly in chunks of 8 and the stop flag is read back after each chunk.
 * Every call on a GPU shares that GPU's array: calls that overlap on one
 * GPU (other streams, other threads) race and must not be made.  The call
 * clears what must start at zero and synchronises before returning.
 * Errors: FVM_EINVAL for another preconditioner, a mixed-precision case, a
 * case too large for the array (the message gives the bytes needed) or a
 * case whose workspace is not on the current device (the array used is the
 * current device's); FVM_EDEVICE when the array's address cannot be
 * obtained. */
fvm_status solve_pressure_static(fvm_case *c, const double *d_gamma_f, const double *d_rhs, double *d_p,
                                 const fvm_solver_ctl *ctl, void *stream, fvm_solve_info *info);

/* fvm_dic_apply -- the diagonal incomplete Cholesky preconditioner alone
 * (diagnostics and tests): assemble the pressure matrix from d_gamma_f as
 * solve_pressure does, factor it (D*_i = A_ii - sum_{j<i} A_ij^2 / D*_j) and
 * apply M^-1 = ((D* + L) D*^-1 (D* + U))^-1 to d_r, giving d_z (and D* in
 * d_dstar unless NULL).  Needs a case created with FVM_PC_DIC.  Overwrites
 * the case's pressure work arrays, not its fields.  Synchronises. */
fvm_status fvm_dic_apply(fvm_case *c, const double *d_gamma_f, const double *d_r, double *d_z, double *d_dstar,
                         void *stream);

/* ---- Comparison layout: the paper's hybrid matrix format (Section 3.1) ----
 * Row i of a mesh's matrix holds the diagonal and one entry per internal
 * face of cell i, in ascending column order.  The first K entries form the
 * ELL part B: values V, columns I, and J, the slot at which the transposed
 * entry sits in B, which gives column access (A^T x) without a transposed
 * copy.  Entries beyond K form the CRS part C.  Face data lives once per
 * face, at the entry of its owner row; the other cell reaches it through I
 * and J.  The solver itself uses the face-major layout; this one exists to
 * compare the two on the same operators. */

/* fvm_mesh_hybrid -- the index arrays of the hybrid layout with K slots per
 * row, in the paper's row-major form (host arrays the caller allocates; any
 * may be NULL): I, J, Q [n_cells * K], c_start [n_cells + 1], c_col and
 * c_tr [n_crs].  Unused slots hold I = i, J = k (value 0).  J = -1 - c when
 * the transposed entry lies at position c of C; c_tr = K * j + k' for a
 * transpose at slot k' of row j in B, else -1 - c'.  Q packs I and J as
 * K * I + J where J >= 0 (-1 elsewhere).  Call with NULL arrays to learn
 * n_crs.  Errors: FVM_EINVAL for K < 1 or K * n_cells beyond int32. */
fvm_status fvm_mesh_hybrid(const fvm_mesh *mesh, int32_t K, int32_t *n_crs, int32_t *I, int32_t *J, int32_t *Q,
                           int32_t *c_start, int32_t *c_col, int32_t *c_tr);

/* fvm_mesh_amg -- the aggregation AMG hierarchy the FVM_PC_AMG
 * preconditioner builds for this mesh (host arrays the caller allocates;
 * any may be NULL): the number of levels, and for `level` its cell and face
 * counts, its faces (own < nei, sorted) and, except on the last level, the
 * aggregate of each cell on the next level.  Level 0 is the mesh, its faces
 * in canonical order.  Errors: FVM_EINVAL for a level out of range. */
fvm_status fvm_mesh_amg(const fvm_mesh *mesh, int32_t level, int32_t *n_levels, int32_t *n_cells, int32_t *n_faces,
                        int32_t *own, int32_t *nei, int32_t *agg);

enum {
    FVM_OP_GRAD = 0, FVM_OP_DIV = 1, FVM_OP_LAP = 2, FVM_OP_SPMV = 3,
    FVM_OP_HY_GRAD = 4, FVM_OP_HY_DIV = 5, FVM_OP_HY_LAP = 6, FVM_OP_HY_SPMV = 7, FVM_OP_HY_STMVP = 8,
    FVM_OP_HY_SETMAT = 9
};

/* fvm_case_operator -- one assembly or matrix operator (Table 3's set), in
 * the face-major layout of the solver (FVM_OP_GRAD .. FVM_OP_SPMV) or in the
 * hybrid layout (FVM_OP_HY_*; the case must have been created with
 * opts.hybrid_K > 0), enqueued on `stream`.  Device arrays, caller order:
 *   GRAD, HY_GRAD: d_in cell scalar [n_cells]; d_out its Gauss gradient
 *     [3][n_cells] (component-major); boundary faces take the case's p
 *     patches (FIXED value, ZERO_GRAD owner value, EMPTY skipped).
 *   DIV, HY_DIV: d_in face flux [n_faces] along the caller's Sf; d_out the
 *     net outward flux of each cell over its non-EMPTY faces [n_cells].
 *   LAP, HY_LAP: d_in gamma [n_faces]; assembles the matrix solve_pressure
 *     builds (face coefficients gamma |S|^2 / (S.d), FIXED-p boundary terms,
 *     the reference pin) into the layout; d_out its diagonal [n_cells]
 *     (LAP) or the layout's values [K * n_cells + n_crs], B slot-major (row
 *     i, slot k at k * n_cells + i) then C (HY_LAP).
 *   SPMV: d_in x [n_cells]; d_out A x with the matrix of the last LAP.
 *   HY_SPMV, HY_STMVP: d_in x; d_out A x or A^T x with the layout's values.
 *   HY_SETMAT: d_in [diag n_cells | upper n_int | lower n_int], upper / lower
 *     per caller internal face = the coefficient in the row of the caller's
 *     owner / neighbour; sets the layout's values.
 * Inputs are first converted into the layout (not part of the operator's
 * profile class).  The case's fields are not touched; its pressure work
 * arrays are.  Errors: FVM_EINVAL for an unknown op, or an FVM_OP_HY_* op on
 * a case without the layout. */
fvm_status fvm_case_operator(fvm_case *c, int32_t op, const double *d_in, double *d_out, void *stream);

/* piso_step_batch -- advance several resident cases by n_steps PISO steps,
 * their kernels batched into shared launches (continuous-batching serving).
 * Every case must be FVM_MIXED or every case FVM_FP64.  When every case
 * qualifies for whole-step kernels (FVM_STEP_AUTO above), one launch runs
 * all n_steps steps of all cases, one workgroup per case, with no host
 * round trip in between; otherwise every case runs launched phases.
 * infos[i] (may be NULL) receives case i's last-step record.  Each case's
 * result is the same as piso_step on it alone. */
fvm_status piso_step_batch(fvm_case *const *cases, int32_t n_cases, int32_t n_steps, void *stream,
                           fvm_step_info *infos);

/* Kernel timing for measurement: while enabled, every launch of a kernel
 * class is bracketed by HIP events on the stream it runs on; read returns the
 * summed device time (ms) and launch count of one class (e.g. "pcg_spmv") and
 * waits for the recorded events.  enable(1) also clears the record. */
fvm_status fvm_profile_enable(int32_t on);
fvm_status fvm_profile_read(const char *kernel_class, double *total_ms, int64_t *launches);

const char *fvm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* FVM_H */
