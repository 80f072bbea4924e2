// Internal declarations shared by the host library and the HIP kernels.
#pragma once

#include <cstddef>
#include <cstdint>
#include <memory>
#include <string>
#include <vector>

#include "fvm.h"

struct fvm_mesh;
struct HybridHost;
// builds h from the canonical mesh (see HybridHost); K >= 1
void build_hybrid(const fvm_mesh &m, int32_t K, HybridHost &h);
struct AmgHost;
// the AMG hierarchy of the mesh's cell graph, built once and cached
const AmgHost &mesh_amg(const fvm_mesh &m);
constexpr int kAmgCoarseMax = 128;    // coarsen while a level has more cells
constexpr int kAmgDenseMax = 512;     // largest coarsest level (dense inverse)
constexpr int kAmgTailLds = 64 * 1024;   // LDS bytes of the fused smallest-levels launch

struct ihipStream_t;
typedef struct ihipStream_t *hipStream_t;

// ---------------------------------------------------------------------------
// Host-side canonical mesh (built by fvm_mesh_create, uploaded per case)
// ---------------------------------------------------------------------------
// The paper's hybrid matrix layout (Section 3.1), built on the host from the
// canonical faces: row i holds its entries in ascending column order (the
// faces seen from the neighbour side, the diagonal, the owned faces); the
// first K go to the ELL part B, the rest to the CRS part C.
//   paper form (row-major, exported for checks): I[i*K+k] column, J[i*K+k]
//   slot of the transposed entry in B, or -1 - c for position c in C; an
//   unused slot holds I = i, J = k.  C: c_start[N+1], c_col, c_tr (K*j+k'
//   for a transpose in B, -1 - c' in C).
//   device form: B slot-major at k*N + i, C after it at K*N + c; dI, dJ as
//   I, J; dpos[i] = position of the diagonal, locO[f] / locN[f] = positions
//   of the owner-side / neighbour-side entries of canonical internal face f;
//   c_trpos = device position of each C entry's transpose.
struct HybridHost {
    int32_t K = 0, nC = 0;
    std::vector<int32_t> I, J, c_start, c_col, c_tr;
    std::vector<int32_t> dI, dJ, dpos, locO, locN, c_trpos;
};

// Aggregation AMG hierarchy of the cell graph (pressure preconditioner).
// Level 0 is the mesh; level l + 1 aggregates level l: agg[l] maps its
// cells to the next level's.  Coarse faces are the distinct aggregate
// pairs joined by a fine face, canonical (lower, upper) and sorted.  The
// gather lists of a coarse level name, per coarse cell, its member cells
// (restriction, diagonal) and the fine faces inside it; per coarse face,
// the fine faces joining its two aggregates; all in ascending fine order.
struct AmgLevelHost {
    int32_t n = 0, nf = 0;
    std::vector<int32_t> own, nei, own_start, nbr_start, losort;   // levels >= 1
    std::vector<int32_t> agg;                                      // [n], all but the last level
    std::vector<int32_t> mstart, members, istart, inner, cstart, cfaces;   // levels >= 1
};
struct AmgHost {
    std::vector<AmgLevelHost> L;
};

struct fvm_mesh {
    int32_t N = 0, F = 0, Fi = 0, Fb = 0, npatch = 0;
    // internal faces in canonical order: own[c] < nei[c], sorted by (own, nei);
    // own[] continues over the boundary faces (caller order) with their cells
    std::vector<int32_t> own, nei;
    std::vector<int32_t> face_user;   // canonical internal face -> caller's face index
    std::vector<int32_t> face_sign;   // +1, or -1 when the caller's orientation is reversed
    std::vector<int32_t> own_start;   // [N+1] faces owned by cell i: [own_start[i], own_start[i+1])
    std::vector<int32_t> nbr_start;   // [N+1] range of losort holding the faces whose neighbour is i
    std::vector<int32_t> losort;      // [Fi] canonical faces ordered by (nei, own)
    std::vector<int32_t> bnd_start;   // [N+1] range of bnd_list holding the boundary faces of cell i
    std::vector<int32_t> bnd_list;    // [Fb] boundary face ids (0-based within the boundary block)
    std::vector<int32_t> bpatch;      // [Fb] patch of each boundary face
    // geometry, structure-of-arrays: x block then y then z
    std::vector<double> S;            // [3*F] canonical orientation (internal), caller order (boundary)
    std::vector<double> Cf;           // [3*F]
    std::vector<double> C;            // [3*N]
    std::vector<double> V;            // [N]
    std::vector<fvm_patch> patches;
    bool nonorth = false;
    bool has_fixed_p = false;
    // level schedule of the lower-triangular dependency graph (DIC sweeps):
    // cells of level l are lvl_cells[lvl_start[l] .. lvl_start[l+1]); lvl_pos
    // is the inverse permutation (position of cell i in lvl_cells), lvl_of the
    // level of each cell
    std::vector<int32_t> lvl_start, lvl_cells, lvl_pos, lvl_of;
    // DIC dependencies in level order: for position q (cell lvl_cells[q]),
    // lower dependency k (ascending neighbour index) at dl_*[k * N + q],
    // upper ones at du_*[k * N + q]; *_pos = position of the neighbour,
    // *_face = its face, -1 past the cell's count
    int32_t dW_lo = 0, dW_hi = 0;
    std::vector<int32_t> dl_pos, dl_face, du_pos, du_face;
    // row-sliced copy of the off-diagonal structure (sliced ELL): slice s =
    // cells [256 s, 256 s + 256), sell_W slots per cell, entry (s, k, lane) at
    // (s * sell_W + k) * 256 + lane; a cell's entries in ascending column.
    // sell_fe: 2 f + 0 for an owned face f (coefficient multiplies the
    // neighbour: upper), 2 f + 1 for a neighbour-side face (lower), -1 for
    // padding.  A slice whose column offsets j - i take at most sell_W
    // values is "regular" (sell_mode 0): slot k holds offset sell_off[s, k]
    // for every cell of the slice and no column is stored; otherwise
    // (sell_mode 1) columns are explicit in sell_col (padding: the cell).
    // sell_mir[s, k] (regular slices, lower slots k): the slot k' that holds
    // the same coefficients in the slices of the neighbours j = i + off_k
    // (offset -off_k there), where the symmetric value a_ji = a_ij can be
    // read instead of the slice's own copy; -1 where that does not hold for
    // every cell of the slice (upper slots, explicit slices, borders).
    int32_t sell_W = 0;
    std::vector<int32_t> sell_mode, sell_off, sell_fe, sell_col, sell_mir;
    // regular slices of the 7-point form the FP64 product takes two cells
    // per thread on: slots (-c, -b, -1, +1, +b, +c), b and c even, lower
    // slots mirrored from the upper ones, every neighbour inside the mesh
    int32_t sell_n7 = 0;
    mutable std::shared_ptr<AmgHost> amg;   // AMG hierarchy, built on first use
};

// ---------------------------------------------------------------------------
// Device-resident Krylov scalars of one linear system.  Written by the last
// block of each reducing kernel, read by the next kernels and by the host.
// ---------------------------------------------------------------------------
struct KState {
    double rho;       // current r.z (CG) / z.r~ (BiCG)
    double beta;
    double alpha;
    double nf;        // residual normalisation
    double tol_eff;   // max(tol, rel_tol * nres0)
    double nres0;
    double nres;
    double xbar;
    double tol, rel_tol;
    double scale;     // mixed precision: scaling of the demoted residual
    double omega;     // BiCGStab
    int32_t iters;
    int32_t done;     // 1: converged / stopped / failed; every iteration kernel is then a no-op
    int32_t status;   // FVM_OK, FVM_WARN_MAXITER, FVM_ENUMERIC
    int32_t max_iter;
    int32_t first;    // 1 before the first direction update
    int32_t half;     // BiCGStab: the half-step residual s passed the stopping test
    int32_t pad[2];
};
static_assert(sizeof(KState) == 128, "KState layout");
// internal status of a mixed-precision momentum component whose FP32 inner
// solve broke down (non-finite value or a zero denominator): the component
// stops its refinement there and continues as an FP64 BiCG solve from the
// current iterate (never reported: the FP64 solve sets the final status)
constexpr int32_t kStatusFallback = 3;

constexpr int kBlock = 256;
constexpr int kGroup = 64;           // blocks per first-level reduction group
constexpr int kMaxRed = 12;          // reduced quantities per kernel
constexpr int kNumKs = 8;            // Krylov states per case

// ---------------------------------------------------------------------------
// Device view of one case: every pointer lies inside the caller's workspace.
// ---------------------------------------------------------------------------
// one level of the AMG hierarchy on the device (level 0 points at the
// case's own topology and pressure matrix; b = the CG residual, out = z)
struct AmgLevel {
    int32_t n, nf;
    const int32_t *own, *nei, *own_start, *nbr_start, *losort, *agg;
    const int32_t *mstart, *members, *istart, *inner, *cstart, *cfaces;
    double *diag, *offd, *x, *b, *r, *out;
};

struct DevCase {
    int32_t N, F, Fi, Fb, npatch;
    int32_t nonorth, has_fixed_p, pin_cell;
    // per-case controls read by the kernels (a launch may serve many cases)
    double nu, dt, alpha_u, alpha_p, p_ref, inner_rel_tol;
    int32_t upwind, inner_max_iter;
    double u_tol, u_rel_tol, p_tol, p_rel_tol;
    int32_t u_max_iter, p_max_iter;
    // topology
    int32_t *own, *nei, *own_start, *nbr_start, *losort, *bnd_start, *bnd_list, *bpatch;
    int32_t *face_user, *face_sign;
    // patches
    int32_t *patch_uk, *patch_pk;
    double *patch_uv, *patch_pv;    // [npatch*3], [npatch]
    // geometry (SoA)
    double *Sx, *Sy, *Sz, *V;
    double *w, *dl, *kx, *ky, *kz;  // w, k: internal faces; dl: all faces
    // fields
    double *U;       // [3][N]
    double *p;       // [N]
    double *phi;     // [F] canonical orientation
    double *p_prev;  // [N]
    double *U_save, *p_save, *phi_save;   // start-of-step copies (rollback)
    // momentum system
    double *mdiag, *upper, *lower, *src, *rhs;   // src, rhs: [3][N]
    double *gradU;   // [9][N] (non-orthogonal meshes)
    double *ns;      // [3][Fi] non-orthogonal momentum source per face
    // pressure corrector
    double *rAU, *HbyA, *gradp, *phiH, *gam, *pdiag, *poff, *pb, *tno;
    // Krylov work vectors
    double *r, *rt, *pp, *pt, *q, *qt;           // [3][N] each (CG uses component 0)
    double *ph, *sh;                             // [3][N] BiCGStab: preconditioned p and s
    int32_t u_stab;                              // momentum solver is BiCGStab
    double *z;                                   // [N] DIC preconditioned residual (cell order)
    double *dstar;                               // [N] DIC diagonal (cell order, for diagnostics)
    int32_t *lvl_cells;                          // DIC level schedule: cells in level order
    int32_t n_levels;
    int32_t dic_lag;                             // DIC sweep gate distance (positions)
    // DIC dependencies in level order (see fvm_mesh), their coefficients
    // (refilled at the start of every solve) and the values published by the
    // sweeps, indexed by level position: D*, y (forward), z (backward)
    int32_t dW_lo, dW_hi;
    int32_t *dl_pos, *dl_face, *du_pos, *du_face;
    double *dl_val, *du_val;
    double *dq, *yq, *zq;
    // sliced-ELL copy of the pressure matrix (structure as in fvm_mesh;
    // sell_mode 2 marks a regular slice whose diagonals the product derives
    // from the coefficients: no fixed-pressure face, no reference pin)
    int32_t sell_W, sell_n7;
    int32_t *sell_mode, *sell_off, *sell_fe, *sell_col, *sell_mir;
    double *sell_val;                            // FP64 values (FP64 cases)
    float *f_sell_val;                           // FP32 values (mixed cases)
    // FP32 copies (mixed precision)
    float *f_diag, *f_up, *f_lo, *f_pdiag, *f_poff;
    float *f_pexc;   // pressure row sums diag_i + sum_f off_f (FP64 sum, rounded)
    float *f_x, *f_b, *f_r, *f_rt, *f_p, *f_pt, *f_q, *f_qt;   // [3][N]
    // the paper's hybrid layout (comparison operators; see HybridHost): B
    // slot-major at k*N + i, C after it at hy_K*N + c; face data (S, w, dl),
    // gamma and flux once per face at the owner-side entry
    int32_t hy_K, hy_nC;
    int32_t *hy_I, *hy_J, *hy_dpos, *hy_locO, *hy_locN, *hy_cstart, *hy_ccol, *hy_ctrpos;
    double *hy_V, *hy_Sx, *hy_Sy, *hy_Sz, *hy_w, *hy_dl, *hy_g, *hy_phi;
    // AMG preconditioner: amg_nl levels (device descriptors), the inverse
    // of the coarsest matrix (amg_nc x amg_nc, row-major)
    int32_t amg_nl, amg_nc;
    int32_t amg_n[20], amg_nf[20];               // level sizes (read by the host launcher)
    AmgLevel *amg;
    double *amg_cinv;
    double *amg_img;                             // [kAmgTailLds / 8] LDS image of the smallest levels
    double *amg_b[20], *amg_out[20];             // each level's right-hand side and result (host copies)
    // reductions
    double *partials;                            // [kMaxRed][red_stride]   level-1 slots
    double *partials2;                           // [kMaxRed][red_stride2]  level-2 slots
    int32_t red_stride, red_stride2;             // >= any reducing grid, and its groups
    unsigned int *gticket;                       // [red_stride2] group tickets
    unsigned int *ticket;
    KState *ks;                                  // [8]: 0..2 momentum, 3 pressure; 4..7 their FP32 inner solves
    // setup temporaries (alias Krylov vectors)
    double *tmpC, *tmpCf;
    KState *ks_gather;                           // [kMaxBatch][kNumKs] staging of a batch's states
    DevCase *self;                               // device copy of this descriptor
};

// ---------------------------------------------------------------------------
// A launch serves up to kMaxBatch cases: block b belongs to the case c with
// start[c] <= b < start[c+1]; every case's block count is a multiple of 8, so
// a block sits on the same XCD (b mod 8) whether its case runs alone or in a
// batch, and each case's reductions see the same partial-sum order.
// ---------------------------------------------------------------------------
constexpr int kMaxBatch = 32;
struct Batch {
    const DevCase *dc[kMaxBatch];
    int32_t start[kMaxBatch + 1];
    int32_t n;
};
// grid kinds: one block per 256 cells / faces / internal faces / max(N, Fi),
// and per 512 / 1024 / 2048 / 4096 cells for kernels that take several cells
// per thread or several slices per block
enum { SZ_CELL = 0, SZ_FACE = 1, SZ_FACEI = 2, SZ_MAXNF = 3, SZ_CELL2 = 4, SZ_CELL4 = 5, SZ_CELL8 = 6, SZ_CELL16 = 7,
       SZ_KINDS = 8 };
struct BatchSet {
    Batch b[SZ_KINDS];
    const DevCase *host[kMaxBatch];   // host copies (sizes, pointers) of the same cases
    int n;
};

// ---------------------------------------------------------------------------
// Launchers (kernels.hip).  All enqueue on `s`; none synchronises.
// ---------------------------------------------------------------------------
int grid_for(int n);
int blocks_for(int n);     // element-wise launches: 256 per block, multiple of 8
void batch_add(BatchSet &bs, const DevCase *dev, const DevCase *host);

// single-case utilities (caller arrays in the caller's numbering)
void launch_geometry(const BatchSet &bs, hipStream_t s);
void launch_flux_from_U(const BatchSet &bs, hipStream_t s);
void launch_U_in(const BatchSet &bs, const double *U_user, hipStream_t s);
void launch_U_out(const BatchSet &bs, double *U_user, hipStream_t s);
void launch_phi_in(const BatchSet &bs, const double *phi_user, hipStream_t s);
void launch_phi_out(const BatchSet &bs, double *phi_user, hipStream_t s);
void launch_gather_faces(const BatchSet &bs, const double *user_face_vals, double *canon, hipStream_t s);
void launch_p_system_from_gamma(const BatchSet &bs, const double *gamma_canon, const double *rhs, hipStream_t s);
void launch_init_partials(const BatchSet &bs, hipStream_t s);
void launch_clear_reduction(const BatchSet &bs, hipStream_t s);   // partials at the sentinel, tickets at 0
// static scratch of solve_pressure_static (kernels.hip): the current
// device's address of the array (looked up once per device), or NULL with
// the HIP error code in *hip_err
constexpr size_t kStaticScratchBytes = (size_t)4 << 20;
void *static_scratch(int *hip_err);
void launch_set_patch(const BatchSet &bs, int patch, double u0, double u1, double u2, double pv, hipStream_t s);

// state save / restore (rollback of a failed step)
void launch_save(const BatchSet &bs, int restore, hipStream_t s);

// momentum assembly: mode 0 PISO (ddt), 1 SIMPLE (relaxed, no ddt)
void launch_gradU(const BatchSet &bs, hipStream_t s);
void launch_mom_face(const BatchSet &bs, hipStream_t s);
void launch_mom_cell(const BatchSet &bs, int mode, hipStream_t s);

// pressure corrector pieces
void launch_hbya(const BatchSet &bs, int with_gradp, hipStream_t s);
void launch_gradp(const BatchSet &bs, hipStream_t s);
void launch_p_face(const BatchSet &bs, hipStream_t s);
void launch_p_cell(const BatchSet &bs, hipStream_t s);
void launch_flux_corr(const BatchSet &bs, hipStream_t s);
void launch_p_relax(const BatchSet &bs, hipStream_t s);
void launch_U_corr(const BatchSet &bs, hipStream_t s);

// Krylov controls: src 0 = the case's momentum controls, 1 = its pressure
// controls, 2 = the explicit values given
void launch_set_ctl(const BatchSet &bs, int first, int count, int src, double tol, double rel_tol, int max_iter,
                    hipStream_t s);
// copy the Krylov states of every case of the batch next to each other
void launch_gather_ks(const BatchSet &bs, hipStream_t s);

// Krylov: momentum BiCG on the three components (FP64)
void launch_bicg_init(const BatchSet &bs, int stab, hipStream_t s);
void launch_bicg_iter(const BatchSet &bs, hipStream_t s);
// Krylov: momentum BiCGStab on the three components (FP64)
void launch_bicgstab_iter(const BatchSet &bs, hipStream_t s);
// Krylov: pressure CG (FP64), Jacobi or DIC
void launch_pcg_init(const BatchSet &bs, int dic, hipStream_t s);
void launch_pcg_iter(const BatchSet &bs, int dic, int parity, hipStream_t s);   // parity: iteration index & 1
void launch_bicg_fallback(const BatchSet &bs, hipStream_t s);   // restart kStatusFallback components as FP64 BiCG
void launch_dic_precond(const BatchSet &bs, int with_setup, hipStream_t s);
void launch_dic_reset(const BatchSet &bs, hipStream_t s);
// mixed precision momentum (restarted FP32 BiCG inside FP64 refinement)
void launch_mx_cvt(const BatchSet &bs, int kind, hipStream_t s);
void launch_mx_inner_init(const BatchSet &bs, int kind, hipStream_t s);
void launch_mx_inner_iter(const BatchSet &bs, int kind, hipStream_t s);
void launch_mx_correct_resid(const BatchSet &bs, int kind, hipStream_t s);
// mixed-precision pressure CG: FP32 recurrence with FP64 residual replacement
void launch_operator(const BatchSet &bs, int op, const double *in, double *out, hipStream_t s);
// AMG preconditioner of the pressure CG (single-case groups): with_setup
// rebuilds the coarse operators and the coarsest inverse; then z = V(r) and
// r.z -> rho, beta
void launch_amg_precond(const BatchSet &bs, int with_setup, hipStream_t s);
void launch_hybrid_geometry(const BatchSet &bs, hipStream_t s);
// whole PISO steps, one workgroup per case (small orthogonal Jacobi/BiCG
// cases, n_corr <= kSoloMaxCorr): grid = the batch's cases; the last
// step's record is left in each case's Krylov state slots (see
// k_solo_piso)
void launch_solo_piso(const BatchSet &bs, int n_steps, int n_corr, hipStream_t s);
constexpr int kSoloMaxCells = 1 << 15;
constexpr int kSoloMaxCorr = kNumKs - 4;
void launch_rr_start(const BatchSet &bs, hipStream_t s);
void launch_rr_iter(const BatchSet &bs, int parity, hipStream_t s);
void launch_rr_replace(const BatchSet &bs, hipStream_t s);

// profiling
void prof_begin(const char *cls, hipStream_t s);
void prof_end(const char *cls, hipStream_t s);

