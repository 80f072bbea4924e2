// HIP kernels (gfx950) of the finite-volume PISO / SIMPLE hot path.
//
// Layout (all device memory in the caller's workspace):
//   * internal faces canonical (own < nei), sorted by (own, nei): the faces a
//     cell owns are the contiguous range own_start[i]..own_start[i+1];
//   * losort lists the same faces ordered by (nei, own): the faces a cell
//     sees from the neighbour side are losort[nbr_start[i]..nbr_start[i+1]];
//   * boundary faces are listed per cell through bnd_start / bnd_list;
//   * vectors of three components are structure-of-arrays [3][N].
// Face quantities are produced once per face by face-parallel kernels
// (coalesced streams over faces) and consumed by cell-parallel gathers; a
// cell sums its faces in a fixed order (owned faces, then neighbour-side
// faces, then boundary faces), so every result is deterministic and no
// floating-point atomics are used.
//
// Batching: every kernel takes a Batch (up to kMaxBatch cases, each with its
// own descriptor in its own workspace); a block first finds its case.  A
// case's block count is a multiple of 8, so a block runs on the same XCD and
// sees the same partial-sum order whether its case is launched alone or
// together with others: results do not depend on the batch.
//
// Work decomposition: a reducing kernel gives each block 256 consecutive
// cells; block b runs on XCD b % 8 and its tile index is remapped so that
// each XCD walks one contiguous eighth of the cells, keeping neighbour
// gathers in the L2 of the XCD that produced them.
//
// Reductions: wave xor-shuffles, LDS across waves, then a two-level grid
// reduction through device-scope atomic slots (no memory fence, see
// reduce_last).  The Krylov scalars live in device memory; a solve never
// synchronises with the host per iteration, and every iteration kernel is a
// no-op once its system is done.
#include <hip/hip_runtime.h>

#include <cmath>
#include <mutex>

#include "fvm_internal.h"

namespace {

constexpr int kWaves = kBlock / 64;
// a NaN payload marks "not yet published" (reduction slots, DIC sweeps)
constexpr unsigned long long kSentinel = 0x7FF8DEADBEEF0001ULL;
constexpr unsigned long long kQNaN = 0x7FF8000000000000ULL;
constexpr int kSpinLimit = 1 << 18;

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

// sentinels are written as integers: a double-typed store of a NaN constant
// need not keep its bit pattern
__device__ __forceinline__ void clear_word(double *a, long i) { reinterpret_cast<unsigned long long *>(a)[i] = kSentinel; }

// ---------------------------------------------------------------------------
// case resolution
// ---------------------------------------------------------------------------
struct Blk {
    const DevCase *d;
    int raw;   // block index within the case
    int lb;    // XCD-remapped tile index within the case
    int G;     // blocks of the case
};

// Blocks are dispatched in index order, round-robin over the 8 XCDs: block
// raw runs on XCD raw % 8, so XCD x takes tiles [x G/8, (x+1) G/8) and keeps
// the same cells in every kernel.  rev = 1 walks each XCD's tiles from the
// last one down: a kernel that follows one walked the other way starts on
// the cells its predecessor touched last, whose lines are the likeliest to
// be still in the memory-side cache.  Only the time order changes: a tile
// covers the same cells and its partial sums take the same slots.
__device__ __forceinline__ Blk resolve(const Batch &b, int rev)
{
    const int bid = blockIdx.x;
    int c = 0;
    while (c + 1 < b.n && bid >= b.start[c + 1]) ++c;
    Blk k;
    k.d = b.dc[c];
    k.raw = bid - b.start[c];
    k.G = b.start[c + 1] - b.start[c];
    if ((k.G & 7) == 0) {
        const int per = k.G >> 3, r = k.raw >> 3;
        k.lb = (k.raw & 7) * per + (rev ? per - 1 - r : r);
    } else k.lb = rev ? k.G - 1 - k.raw : k.raw;
    return k;
}

#define CASE_OF(bt)                \
    const Blk K = resolve(bt, 0);  \
    const DevCase &d = *K.d

// the same, walking the tiles in the direction rev
#define CASE_OF_DIR(bt, rev)         \
    const Blk K = resolve(bt, rev);  \
    const DevCase &d = *K.d

struct Range {
    int beg, end;
};

__device__ __forceinline__ Range block_range(int n, const Blk &K)
{
    long per = ((long)n + K.G - 1) / K.G;
    per = (per + kBlock - 1) / kBlock * kBlock;
    const long b = (long)K.lb * per;
    Range r;
    r.beg = (int)(b < n ? b : n);
    r.end = (int)(b + per < n ? b + per : n);
    return r;
}

// ---------------------------------------------------------------------------
// reductions
// ---------------------------------------------------------------------------
template <int NV>
__device__ __forceinline__ void wave_sum(double (&v)[NV])
{
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
}

// fixed-order block sum of NV values; result valid in thread 0
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (&lds)[NV][kWaves])
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    wave_sum(v);
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[k][wv] = v[k];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = lds[k][0];
            for (int w = 1; w < kWaves; ++w) s += lds[k][w];
            v[k] = s;
        }
}

// Global-address-space view of a device pointer.  Accesses through it are
// global rather than flat: a flat access also counts against the counter
// that scalar-memory and LDS accesses share, so a wait for a scalar load or
// an LDS value also waits for it, and a wait for one flat load is a wait for
// all of them.
template <class T>
__device__ __forceinline__ __attribute__((address_space(1))) T *gmem(T *p)
{
    return (__attribute__((address_space(1))) T *)p;
}

// Slots hold the NaN sentinel while empty.  A device-scope release fence
// would compile to a write-back of the whole L2 of the XCD; instead each
// value is published by one device-scope atomic store, and the reader waits
// on the slot itself, then refills it with the sentinel.
// device-scope accesses through global-address-space pointers (a flat
// access would also wait on the LDS counter)
typedef __attribute__((address_space(1))) unsigned long long gword;
__device__ __forceinline__ unsigned long long gld(const void *a)
{
    return __hip_atomic_load((const gword *)a, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void gst(void *a, unsigned long long v)
{
    __hip_atomic_store((gword *)a, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// take NV published slots slot + k * stride (all loads issued before the
// first comparison), re-arming each with the sentinel
template <int NV>
__device__ __forceinline__ void slots_take(double *slot, int stride, double (&out)[NV])
{
    unsigned long long b[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) b[k] = gld(slot + (long)k * stride);
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        for (int spin = 0; b[k] == kSentinel && spin < kSpinLimit; ++spin) {
            __builtin_amdgcn_s_sleep(1);
            b[k] = gld(slot + (long)k * stride);
        }
        gst(slot + (long)k * stride, kSentinel);
        out[k] = b[k] == kSentinel ? __longlong_as_double((long long)kQNaN) : __longlong_as_double((long long)b[k]);
    }
}

__device__ __forceinline__ void slot_put(double *slot, double v)
{
    unsigned long long b = (unsigned long long)__double_as_longlong(v);
    if (b == kSentinel) b = kQNaN;
    gst(slot, b);
}

// Two-level grid reduction.  Level 1: each block publishes its partials and
// takes its group's ticket (groups of kGroup consecutive tiles); the block
// that completes a group sums the group's slots in order and publishes one
// level-2 partial.  Level 2: the block that completes the last group sums
// the level-2 slots in order.  Returns true in every thread of that final
// block, with the totals in tot[].
template <int NV>
__device__ bool reduce_last(double (&v)[NV], const DevCase &d, const Blk &K, double *tot)
{
    __shared__ double lds[NV][kWaves];
    __shared__ int stage;
    const int G = K.G, lb = K.lb;
    const int grp = lb / kGroup, ngrp = (G + kGroup - 1) / kGroup;
    const int gsize = min(kGroup, G - grp * kGroup);
    block_sum(v, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) slot_put(&d.partials[k * d.red_stride + lb], v[k]);
        const unsigned int t = __hip_atomic_fetch_add(&d.gticket[grp], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        stage = t == (unsigned int)gsize - 1;
    }
    __syncthreads();
    if (!stage) return false;
    double g[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) g[k] = 0.0;
    if ((int)threadIdx.x < gsize) slots_take<NV>(&d.partials[grp * kGroup + threadIdx.x], d.red_stride, g);
    block_sum(g, lds);
    if (threadIdx.x == 0) {
        __hip_atomic_store(&d.gticket[grp], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
        for (int k = 0; k < NV; ++k) slot_put(&d.partials2[k * d.red_stride2 + grp], g[k]);
        const unsigned int t = __hip_atomic_fetch_add(d.ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        stage = t == (unsigned int)ngrp - 1 ? 2 : 0;
    }
    __syncthreads();
    if (stage != 2) return false;
    double a[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) a[k] = 0.0;
    for (int j = threadIdx.x; j < ngrp; j += kBlock) {
        double t[NV];
        slots_take<NV>(&d.partials2[j], d.red_stride2, t);
#pragma unroll
        for (int k = 0; k < NV; ++k) a[k] += t[k];
    }
    block_sum(a, lds);
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) tot[k] = a[k];
        __hip_atomic_store(d.ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    return true;
}

// ---------------------------------------------------------------------------
// gathers
// ---------------------------------------------------------------------------

// y_i = diag_i x_i + sum_owned up_f x_nei + sum_nbrside lo_f x_own.  The
// sum is formed in FP64 for FP32 data too: products of two FP32 values are
// exact in FP64, and an FP32 sum of the nearly cancelling Laplacian terms
// would lose the smooth modes Krylov methods converge on last.
template <class T>
__device__ __forceinline__ T row_apply(const DevCase &d, int i, const T *__restrict__ diag, const T *__restrict__ up,
                                       const T *__restrict__ lo, const T *__restrict__ x)
{
    double acc = (double)diag[i] * (double)x[i];
    const int f0 = d.own_start[i], f1 = d.own_start[i + 1];
    for (int f = f0; f < f1; ++f) acc += (double)up[f] * (double)x[d.nei[f]];
    const int k0 = d.nbr_start[i], k1 = d.nbr_start[i + 1];
    for (int k = k0; k < k1; ++k) {
        const int f = d.losort[k];
        acc += (double)lo[f] * (double)x[d.own[f]];
    }
    return (T)acc;
}

// row sum of the off-diagonal coefficients plus the diagonal (A 1)_i
__device__ __forceinline__ double row_sum(const DevCase &d, int i, const double *__restrict__ diag,
                                          const double *__restrict__ up, const double *__restrict__ lo)
{
    double acc = diag[i];
    for (int f = d.own_start[i]; f < d.own_start[i + 1]; ++f) acc += up[f];
    for (int k = d.nbr_start[i]; k < d.nbr_start[i + 1]; ++k) acc += lo[d.losort[k]];
    return acc;
}

// Gauss gradient sum of a cell scalar x (sum S phi_f, not divided by V), with
// the boundary rule of kinds/vals: FIXED value, ZERO_GRAD owner value, EMPTY
// skipped
__device__ __forceinline__ void gauss_sum(const DevCase &d, int i, const double *__restrict__ x,
                                          const int32_t *__restrict__ kinds, const double *__restrict__ vals,
                                          int vstride, double &g0, double &g1, double &g2)
{
    const double xi = x[i];
    g0 = g1 = g2 = 0.0;
    for (int f = d.own_start[i]; f < d.own_start[i + 1]; ++f) {
        const double w = d.w[f];
        const double pf = w * xi + (1.0 - w) * x[d.nei[f]];
        g0 += d.Sx[f] * pf; g1 += d.Sy[f] * pf; g2 += d.Sz[f] * pf;
    }
    for (int k = d.nbr_start[i]; k < d.nbr_start[i + 1]; ++k) {
        const int f = d.losort[k];
        const double w = d.w[f];
        const double pf = w * x[d.own[f]] + (1.0 - w) * xi;
        g0 -= d.Sx[f] * pf; g1 -= d.Sy[f] * pf; g2 -= d.Sz[f] * pf;
    }
    for (int k = d.bnd_start[i]; k < d.bnd_start[i + 1]; ++k) {
        const int b = d.bnd_list[k], f = d.Fi + b, pt = d.bpatch[b], kind = kinds[pt];
        if (kind == FVM_BC_EMPTY) continue;
        const double pf = kind == FVM_BC_FIXED ? vals[vstride * pt] : xi;
        g0 += d.Sx[f] * pf; g1 += d.Sy[f] * pf; g2 += d.Sz[f] * pf;
    }
}

// ---------------------------------------------------------------------------
// Setup and state exchange
// ---------------------------------------------------------------------------

// w = S.(C_N - Cf)/(S.d), dl = |S|^2/(S.d), k = S - dl d (internal);
// dl_b = |S|^2/(S.(Cf - C_P)) (boundary)
__global__ void k_geometry(Batch bt)
{
    CASE_OF(bt);
    const int f = K.raw * kBlock + threadIdx.x;
    if (f >= d.F) return;
    const double *C = d.tmpC, *Cf = d.tmpCf;
    const long N = d.N, F = d.F;
    const double S0 = d.Sx[f], S1 = d.Sy[f], S2 = d.Sz[f];
    const double SS = S0 * S0 + S1 * S1 + S2 * S2;
    if (f < d.Fi) {
        const int P = d.own[f], Q = d.nei[f];
        const double d0 = C[Q] - C[P], d1 = C[N + Q] - C[N + P], d2 = C[2 * N + Q] - C[2 * N + P];
        const double Sd = S0 * d0 + S1 * d1 + S2 * d2;
        const double n0 = C[Q] - Cf[f], n1 = C[N + Q] - Cf[F + f], n2 = C[2 * N + Q] - Cf[2 * F + f];
        d.w[f] = (S0 * n0 + S1 * n1 + S2 * n2) / Sd;
        const double dl = SS / Sd;
        d.dl[f] = dl;
        if (d.nonorth) {
            d.kx[f] = S0 - dl * d0;
            d.ky[f] = S1 - dl * d1;
            d.kz[f] = S2 - dl * d2;
        }
    } else {
        const int P = d.own[f];
        const double d0 = Cf[f] - C[P], d1 = Cf[F + f] - C[N + P], d2 = Cf[2 * F + f] - C[2 * N + P];
        d.dl[f] = SS / (S0 * d0 + S1 * d1 + S2 * d2);
    }
}

// phi = S.(w U_P + (1-w) U_N) internal; FIXED S.U_b, ZERO_GRAD S.U_P, EMPTY 0
__global__ void k_flux_from_U(Batch bt)
{
    CASE_OF(bt);
    const int f = K.raw * kBlock + threadIdx.x;
    if (f >= d.F) return;
    const long N = d.N;
    const double *U = d.U;
    double v0, v1, v2;
    if (f < d.Fi) {
        const int P = d.own[f], Q = d.nei[f];
        const double w = d.w[f];
        v0 = w * U[P] + (1.0 - w) * U[Q];
        v1 = w * U[N + P] + (1.0 - w) * U[N + Q];
        v2 = w * U[2 * N + P] + (1.0 - w) * U[2 * N + Q];
    } else {
        const int b = f - d.Fi, P = d.own[f], pt = d.bpatch[b], k = d.patch_uk[pt];
        if (k == FVM_BC_FIXED) {
            v0 = d.patch_uv[3 * pt]; v1 = d.patch_uv[3 * pt + 1]; v2 = d.patch_uv[3 * pt + 2];
        } else if (k == FVM_BC_ZERO_GRAD) {
            v0 = U[P]; v1 = U[N + P]; v2 = U[2 * N + P];
        } else {
            d.phi[f] = 0.0;
            return;
        }
    }
    d.phi[f] = d.Sx[f] * v0 + d.Sy[f] * v1 + d.Sz[f] * v2;
}

__global__ void k_U_in(Batch bt, const double *__restrict__ Uu)
{
    CASE_OF(bt);
    const int i = K.raw * kBlock + threadIdx.x;
    if (i >= d.N) return;
    d.U[i] = Uu[3 * (size_t)i];
    d.U[d.N + i] = Uu[3 * (size_t)i + 1];
    d.U[2 * (size_t)d.N + i] = Uu[3 * (size_t)i + 2];
}

__global__ void k_U_out(Batch bt, double *__restrict__ Uu)
{
    CASE_OF(bt);
    const int i = K.raw * kBlock + threadIdx.x;
    if (i >= d.N) return;
    Uu[3 * (size_t)i] = d.U[i];
    Uu[3 * (size_t)i + 1] = d.U[d.N + i];
    Uu[3 * (size_t)i + 2] = d.U[2 * (size_t)d.N + i];
}

__global__ void k_phi_in(Batch bt, const double *__restrict__ pu)
{
    CASE_OF(bt);
    const int f = K.raw * kBlock + threadIdx.x;
    if (f >= d.F) return;
    d.phi[f] = f < d.Fi ? (double)d.face_sign[f] * pu[d.face_user[f]] : pu[f];
}

__global__ void k_phi_out(Batch bt, double *__restrict__ pu)
{
    CASE_OF(bt);
    const int f = K.raw * kBlock + threadIdx.x;
    if (f >= d.F) return;
    if (f < d.Fi) pu[d.face_user[f]] = (double)d.face_sign[f] * d.phi[f];
    else pu[f] = d.phi[f];
}

// caller face order -> canonical order (orientation-free face values)
__global__ void k_gather_faces(Batch bt, const double *__restrict__ uv, double *__restrict__ out)
{
    CASE_OF(bt);
    const int f = K.raw * kBlock + threadIdx.x;
    if (f >= d.F) return;
    out[f] = f < d.Fi ? uv[d.face_user[f]] : uv[f];
}

// start-of-step copies of U, p, phi (restore = 1 copies back)
__global__ void k_save(Batch bt, int restore)
{
    CASE_OF(bt);
    const long t = (long)K.raw * kBlock + threadIdx.x;
    const long N = d.N, F = d.F;
    if (t < 3 * N) {
        if (restore) d.U[t] = d.U_save[t];
        else d.U_save[t] = d.U[t];
    } else if (t < 4 * N) {
        if (restore) d.p[t - 3 * N] = d.p_save[t - 3 * N];
        else d.p_save[t - 3 * N] = d.p[t - 3 * N];
    } else if (t < 4 * N + F) {
        if (restore) d.phi[t - 4 * N] = d.phi_save[t - 4 * N];
        else d.phi_save[t - 4 * N] = d.phi[t - 4 * N];
    }
}

__global__ void k_fill_sentinel(Batch bt)
{
    CASE_OF(bt);
    const long t = (long)K.raw * kBlock + threadIdx.x;
    const long n1 = (long)kMaxRed * d.red_stride, n2 = (long)kMaxRed * d.red_stride2;
    for (long i = t; i < n1; i += (long)K.G * kBlock) clear_word(d.partials, i);
    for (long i = t; i < n2; i += (long)K.G * kBlock) clear_word(d.partials2, i);
}

// reduction slots of a descriptor whose slots live in the static scratch:
// partials at the sentinel, tickets at zero (every call clears them: the
// array keeps the previous call's contents)
__global__ void k_clear_reduction(Batch bt)
{
    CASE_OF(bt);
    const long t = (long)K.raw * kBlock + threadIdx.x, stride = (long)K.G * kBlock;
    const long n1 = (long)kMaxRed * d.red_stride, n2 = (long)kMaxRed * d.red_stride2;
    for (long i = t; i < n1; i += stride) clear_word(d.partials, i);
    for (long i = t; i < n2; i += stride) clear_word(d.partials2, i);
    for (long i = t; i < d.red_stride2; i += stride) d.gticket[i] = 0u;
    for (long i = t; i < 64; i += stride) d.ticket[i] = 0u;
}

__global__ void k_set_patch(Batch bt, int pt, double u0, double u1, double u2, double pv)
{
    CASE_OF(bt);
    if (K.raw != 0 || threadIdx.x != 0) return;
    d.patch_uv[3 * pt] = u0;
    d.patch_uv[3 * pt + 1] = u1;
    d.patch_uv[3 * pt + 2] = u2;
    d.patch_pv[pt] = pv;
}

// ---------------------------------------------------------------------------
// Momentum assembly
// ---------------------------------------------------------------------------

// gradU[3c + k][i] = d U_c / d x_k (start-of-step U; non-orthogonal meshes)
__global__ void k_gradU(Batch bt)
{
    CASE_OF(bt);
    const int i = K.raw * kBlock + threadIdx.x;
    if (i >= d.N || !d.nonorth) return;
    const long N = d.N;
    for (int c = 0; c < 3; ++c) {
        double g0, g1, g2;
        gauss_sum(d, i, d.U + c * N, d.patch_uk, d.patch_uv + c, 3, g0, g1, g2);
        const double V = d.V[i];
        d.gradU[(3 * c) * N + i] = g0 / V;
        d.gradU[(3 * c + 1) * N + i] = g1 / V;
        d.gradU[(3 * c + 2) * N + i] = g2 / V;
    }
}

// upper = F(1-w) - nu dl, lower = -F w - nu dl; non-orthogonal source
// ns_c = nu k.(w gradU_c,P + (1-w) gradU_c,N)
__device__ __forceinline__ void el_mom_face(const DevCase &d, int f)
{
    const double nu = d.nu;
    const double Fl = d.phi[f];
    const double w = d.upwind ? (Fl >= 0.0 ? 1.0 : 0.0) : d.w[f];
    const double D = nu * d.dl[f];
    d.upper[f] = Fl * (1.0 - w) - D;
    d.lower[f] = -Fl * w - D;
    if (d.nonorth) {
        const long N = d.N;
        const int P = d.own[f], Q = d.nei[f];
        const double wi = d.w[f];
        const double k0 = d.kx[f], k1 = d.ky[f], k2 = d.kz[f];
        for (int c = 0; c < 3; ++c) {
            const double *g = d.gradU + (3 * c) * N;
            const double a0 = wi * g[P] + (1.0 - wi) * g[Q];
            const double a1 = wi * g[N + P] + (1.0 - wi) * g[N + Q];
            const double a2 = wi * g[2 * N + P] + (1.0 - wi) * g[2 * N + Q];
            d.ns[(long)c * d.Fi + f] = nu * (k0 * a0 + k1 * a1 + k2 * a2);
        }
    }
}

__global__ void k_mom_face(Batch bt)
{
    CASE_OF(bt);
    const int f = K.raw * kBlock + threadIdx.x;
    if (f >= d.Fi) return;
    el_mom_face(d, f);
}

// diag, src (without the pressure gradient) and rhs = src - V grad p.
// mode 0 (PISO): transient term V/dt, V U/dt.  mode 1 (SIMPLE): implicit
// relaxation diag <- diag/alpha_u, src += (1-alpha_u)/alpha_u diag_orig U.
__device__ __forceinline__ void el_mom_cell(const DevCase &d, int i, int mode)
{
    const long N = d.N;
    const double nu = d.nu;
    const int upwind = d.upwind;
    const double V = d.V[i];
    const double U0 = d.U[i], U1 = d.U[N + i], U2 = d.U[2 * N + i];
    double dg = 0.0, s0 = 0.0, s1 = 0.0, s2 = 0.0;
    if (mode == 0) {
        const double dt = d.dt;
        dg = V / dt;
        s0 = V * U0 / dt; s1 = V * U1 / dt; s2 = V * U2 / dt;
    }
    const double pi = d.p[i];
    double g0 = 0.0, g1 = 0.0, g2 = 0.0;
    for (int f = d.own_start[i]; f < d.own_start[i + 1]; ++f) {
        const double Fl = d.phi[f];
        const double w = d.w[f];
        const double we = upwind ? (Fl >= 0.0 ? 1.0 : 0.0) : w;
        dg += Fl * we + nu * d.dl[f];
        const double pf = w * pi + (1.0 - w) * d.p[d.nei[f]];
        g0 += d.Sx[f] * pf; g1 += d.Sy[f] * pf; g2 += d.Sz[f] * pf;
        if (d.nonorth) {
            s0 += d.ns[f]; s1 += d.ns[(long)d.Fi + f]; s2 += d.ns[2 * (long)d.Fi + f];
        }
    }
    for (int k = d.nbr_start[i]; k < d.nbr_start[i + 1]; ++k) {
        const int f = d.losort[k];
        const double Fl = d.phi[f];
        const double w = d.w[f];
        const double we = upwind ? (Fl >= 0.0 ? 1.0 : 0.0) : w;
        dg += -Fl * (1.0 - we) + nu * d.dl[f];
        const double pf = w * d.p[d.own[f]] + (1.0 - w) * pi;
        g0 -= d.Sx[f] * pf; g1 -= d.Sy[f] * pf; g2 -= d.Sz[f] * pf;
        if (d.nonorth) {
            s0 -= d.ns[f]; s1 -= d.ns[(long)d.Fi + f]; s2 -= d.ns[2 * (long)d.Fi + f];
        }
    }
    for (int k = d.bnd_start[i]; k < d.bnd_start[i + 1]; ++k) {
        const int b = d.bnd_list[k], f = d.Fi + b, pt = d.bpatch[b];
        const double Fl = d.phi[f];
        const int uk = d.patch_uk[pt], pk = d.patch_pk[pt];
        if (uk == FVM_BC_FIXED) {
            const double D = nu * d.dl[f];
            dg += D;
            s0 += (D - Fl) * d.patch_uv[3 * pt];
            s1 += (D - Fl) * d.patch_uv[3 * pt + 1];
            s2 += (D - Fl) * d.patch_uv[3 * pt + 2];
        } else if (uk == FVM_BC_ZERO_GRAD) {
            dg += Fl;
        }
        if (pk != FVM_BC_EMPTY) {
            const double pf = pk == FVM_BC_FIXED ? d.patch_pv[pt] : pi;
            g0 += d.Sx[f] * pf; g1 += d.Sy[f] * pf; g2 += d.Sz[f] * pf;
        }
    }
    if (mode == 1) {
        const double a = d.alpha_u;
        const double d0 = dg;
        dg = d0 / a;
        const double c = (1.0 - a) / a * d0;
        s0 += c * U0; s1 += c * U1; s2 += c * U2;
    }
    d.mdiag[i] = dg;
    d.src[i] = s0; d.src[N + i] = s1; d.src[2 * N + i] = s2;
    d.rhs[i] = s0 - V * (g0 / V);
    d.rhs[N + i] = s1 - V * (g1 / V);
    d.rhs[2 * N + i] = s2 - V * (g2 / V);
}

__global__ void k_mom_cell(Batch bt, int mode)
{
    CASE_OF(bt);
    const int i = K.raw * kBlock + threadIdx.x;
    if (i >= d.N) return;
    el_mom_cell(d, i, mode);
}

// ---------------------------------------------------------------------------
// Pressure corrector
// ---------------------------------------------------------------------------

// H = src - sum a_PN U_N, rAU = V/a_PP, HbyA = H/a_PP; optional grad p
__device__ __forceinline__ void el_hbya(const DevCase &d, int i, int with_gradp)
{
    const long N = d.N;
    double h0 = d.src[i], h1 = d.src[N + i], h2 = d.src[2 * N + i];
    const double *U = d.U;
    for (int f = d.own_start[i]; f < d.own_start[i + 1]; ++f) {
        const int j = d.nei[f];
        const double a = d.upper[f];
        h0 -= a * U[j]; h1 -= a * U[N + j]; h2 -= a * U[2 * N + j];
    }
    for (int k = d.nbr_start[i]; k < d.nbr_start[i + 1]; ++k) {
        const int f = d.losort[k], j = d.own[f];
        const double a = d.lower[f];
        h0 -= a * U[j]; h1 -= a * U[N + j]; h2 -= a * U[2 * N + j];
    }
    const double dg = d.mdiag[i];
    d.rAU[i] = d.V[i] / dg;
    d.HbyA[i] = h0 / dg; d.HbyA[N + i] = h1 / dg; d.HbyA[2 * N + i] = h2 / dg;
    if (with_gradp && d.nonorth) {
        double g0, g1, g2;
        gauss_sum(d, i, d.p, d.patch_pk, d.patch_pv, 1, g0, g1, g2);
        const double V = d.V[i];
        d.gradp[i] = g0 / V; d.gradp[N + i] = g1 / V; d.gradp[2 * N + i] = g2 / V;
    }
}

__global__ void k_hbya(Batch bt, int with_gradp)
{
    CASE_OF(bt);
    const int i = K.raw * kBlock + threadIdx.x;
    if (i >= d.N) return;
    el_hbya(d, i, with_gradp);
}

__global__ void k_gradp(Batch bt)
{
    CASE_OF(bt);
    const int i = K.raw * kBlock + threadIdx.x;
    if (i >= d.N) return;
    double g0, g1, g2;
    gauss_sum(d, i, d.p, d.patch_pk, d.patch_pv, 1, g0, g1, g2);
    const double V = d.V[i];
    d.gradp[i] = g0 / V; d.gradp[d.N + i] = g1 / V; d.gradp[2 * (long)d.N + i] = g2 / V;
}

// face pass: phiH = S.interp(HbyA) (boundary per U kind), gam = interp(rAU)
// (boundary rAU_P), poff = -gam dl, tno = gam k.interp(grad p)
__device__ __forceinline__ void el_p_face(const DevCase &d, int f)
{
    const long N = d.N;
    const double *H = d.HbyA;
    if (f < d.Fi) {
        const int P = d.own[f], Q = d.nei[f];
        const double w = d.w[f];
        const double v0 = w * H[P] + (1.0 - w) * H[Q];
        const double v1 = w * H[N + P] + (1.0 - w) * H[N + Q];
        const double v2 = w * H[2 * N + P] + (1.0 - w) * H[2 * N + Q];
        d.phiH[f] = d.Sx[f] * v0 + d.Sy[f] * v1 + d.Sz[f] * v2;
        const double gm = w * d.rAU[P] + (1.0 - w) * d.rAU[Q];
        d.gam[f] = gm;
        d.poff[f] = -(gm * d.dl[f]);
        if (d.nonorth) {
            const double *g = d.gradp;
            const double a0 = w * g[P] + (1.0 - w) * g[Q];
            const double a1 = w * g[N + P] + (1.0 - w) * g[N + Q];
            const double a2 = w * g[2 * N + P] + (1.0 - w) * g[2 * N + Q];
            d.tno[f] = gm * (d.kx[f] * a0 + d.ky[f] * a1 + d.kz[f] * a2);
        }
    } else {
        const int b = f - d.Fi, P = d.own[f], pt = d.bpatch[b], uk = d.patch_uk[pt];
        double ph = 0.0;
        if (uk == FVM_BC_FIXED)
            ph = d.Sx[f] * d.patch_uv[3 * pt] + d.Sy[f] * d.patch_uv[3 * pt + 1] + d.Sz[f] * d.patch_uv[3 * pt + 2];
        else if (uk == FVM_BC_ZERO_GRAD)
            ph = d.Sx[f] * H[P] + d.Sy[f] * H[N + P] + d.Sz[f] * H[2 * N + P];
        d.phiH[f] = ph;
        d.gam[f] = d.rAU[P];
    }
}

__global__ void k_p_face(Batch bt)
{
    CASE_OF(bt);
    const int f = K.raw * kBlock + threadIdx.x;
    if (f >= d.F) return;
    el_p_face(d, f);
}

// cell pass: pdiag, pb (divergence, fixed-p terms, non-orthogonal part), pin.
// with_div = 0: the stand-alone pressure system (pb holds the given rhs)
__device__ __forceinline__ void el_p_cell(const DevCase &d, int i, int with_div)
{
    double dg = 0.0, b = 0.0;
    for (int f = d.own_start[i]; f < d.own_start[i + 1]; ++f) {
        dg += -d.poff[f];
        if (with_div) b -= d.phiH[f];
        if (d.nonorth && with_div) b += d.tno[f];
    }
    for (int k = d.nbr_start[i]; k < d.nbr_start[i + 1]; ++k) {
        const int f = d.losort[k];
        dg += -d.poff[f];
        if (with_div) b += d.phiH[f];
        if (d.nonorth && with_div) b -= d.tno[f];
    }
    for (int k = d.bnd_start[i]; k < d.bnd_start[i + 1]; ++k) {
        const int bb = d.bnd_list[k], f = d.Fi + bb, pt = d.bpatch[bb], pk = d.patch_pk[pt];
        if (pk == FVM_BC_EMPTY) continue;
        if (with_div) b -= d.phiH[f];
        if (pk == FVM_BC_FIXED) {
            const double g = d.gam[f] * d.dl[f];
            dg += g;
            b += g * d.patch_pv[pt];
        }
    }
    if (i == d.pin_cell && !d.has_fixed_p) {
        const double a = dg;
        dg = 2.0 * a;
        b += a * d.p_ref;
    }
    d.pdiag[i] = dg;
    if (with_div) d.pb[i] = b;
    else d.pb[i] += b;
}

__global__ void k_p_cell(Batch bt, int with_div)
{
    CASE_OF(bt);
    const int i = K.raw * kBlock + threadIdx.x;
    if (i >= d.N) return;
    el_p_cell(d, i, with_div);
}

// gamma given per face (canonical order) -> poff, gam
__global__ void k_p_face_gamma(Batch bt, const double *__restrict__ gam)
{
    CASE_OF(bt);
    const int f = K.raw * kBlock + threadIdx.x;
    if (f >= d.F) return;
    const double g = gam[f];
    d.gam[f] = g;
    if (f < d.Fi) d.poff[f] = -(g * d.dl[f]);
}

// phi = phiH - g (p_N - p_P) - tno (internal); p FIXED: phiH - g_b (p_b - p_P)
__device__ __forceinline__ void el_flux_corr(const DevCase &d, int f)
{
    if (f < d.Fi) {
        double v = d.phiH[f] - d.gam[f] * d.dl[f] * (d.p[d.nei[f]] - d.p[d.own[f]]);
        if (d.nonorth) v -= d.tno[f];
        d.phi[f] = v;
    } else {
        const int b = f - d.Fi, pt = d.bpatch[b];
        if (d.patch_pk[pt] == FVM_BC_FIXED)
            d.phi[f] = d.phiH[f] - d.gam[f] * d.dl[f] * (d.patch_pv[pt] - d.p[d.own[f]]);
        else
            d.phi[f] = d.phiH[f];
    }
}

__global__ void k_flux_corr(Batch bt)
{
    CASE_OF(bt);
    const int f = K.raw * kBlock + threadIdx.x;
    if (f >= d.F) return;
    el_flux_corr(d, f);
}

__global__ void k_p_relax(Batch bt)
{
    CASE_OF(bt);
    const int i = K.raw * kBlock + threadIdx.x;
    if (i >= d.N) return;
    d.p[i] = d.p_prev[i] + d.alpha_p * (d.p[i] - d.p_prev[i]);
}

// U = HbyA - rAU grad p (new p)
__device__ __forceinline__ void el_U_corr(const DevCase &d, int i)
{
    const long N = d.N;
    double g0, g1, g2;
    gauss_sum(d, i, d.p, d.patch_pk, d.patch_pv, 1, g0, g1, g2);
    const double V = d.V[i], r = d.rAU[i];
    d.U[i] = d.HbyA[i] - r * (g0 / V);
    d.U[N + i] = d.HbyA[N + i] - r * (g1 / V);
    d.U[2 * N + i] = d.HbyA[2 * N + i] - r * (g2 / V);
}

__global__ void k_U_corr(Batch bt)
{
    CASE_OF(bt);
    const int i = K.raw * kBlock + threadIdx.x;
    if (i >= d.N) return;
    el_U_corr(d, i);
}

// ---------------------------------------------------------------------------
// Krylov solvers (Barrett et al., "Templates": CG and BiCG)
//
// The iteration kernels are templated on the vector/matrix value type: the
// FP64 solves and the FP32 inner solves of the mixed-precision modes run the
// same code over different arrays.  Every dot product and residual sum is
// accumulated in FP64 whatever the vector type.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void set_done(KState &s, int status)
{
    s.status = status;
    s.done = 1;
}

// array selectors: a view names which arrays of the case a kernel uses
enum { V_FP64 = 0, V_FP32 = 1 };

template <class T>
struct CGArr {
    const T *diag, *off;
    const T *exc;    // FP32 only: row sums, for the difference form of A p
    const T *sval;   // sliced-ELL off-diagonal values
    T *x, *r, *p, *q;
    const double *z;
    KState *ks;
};

template <class T>
__device__ __forceinline__ CGArr<T> cg_arrays(const DevCase &d, int dic);

template <>
__device__ __forceinline__ CGArr<double> cg_arrays<double>(const DevCase &d, int dic)
{
    return CGArr<double>{d.pdiag, d.poff, nullptr, d.sell_val, d.p, d.r, d.pp, d.q, dic ? d.z : nullptr, d.ks + 3};
}

// FP32 recurrence of the mixed-precision pressure CG (x is FP64: not here)
template <>
__device__ __forceinline__ CGArr<float> cg_arrays<float>(const DevCase &d, int)
{
    return CGArr<float>{d.f_pdiag, d.f_poff, d.f_pexc, d.f_sell_val, d.f_x, d.f_r, d.f_p, d.f_q, nullptr, d.ks + 3};
}

template <class T>
struct BiArr {
    const T *diag, *up, *lo;
    T *x, *r, *rt, *p, *pt, *q, *qt;
    KState *ks;
};

template <class T>
__device__ __forceinline__ BiArr<T> bi_arrays(const DevCase &d);

template <>
__device__ __forceinline__ BiArr<double> bi_arrays<double>(const DevCase &d)
{
    return BiArr<double>{d.mdiag, d.upper, d.lower, d.U, d.r, d.rt, d.pp, d.pt, d.q, d.qt, d.ks};
}

template <>
__device__ __forceinline__ BiArr<float> bi_arrays<float>(const DevCase &d)
{
    return BiArr<float>{d.f_diag, d.f_up, d.f_lo, d.f_x, d.f_r, d.f_rt, d.f_p, d.f_pt, d.f_q, d.f_qt, d.ks + 4};
}

// ---- controls ----------------------------------------------------------

__global__ void k_set_ctl(Batch bt, int first, int count, int src, double tol, double rel_tol, int max_iter)
{
    CASE_OF(bt);
    const int k = threadIdx.x;
    if (K.raw != 0 || k >= count) return;
    KState &s = d.ks[first + k];
    if (src == 0) { s.tol = d.u_tol; s.rel_tol = d.u_rel_tol; s.max_iter = d.u_max_iter; }
    else if (src == 1) { s.tol = d.p_tol; s.rel_tol = d.p_rel_tol; s.max_iter = d.p_max_iter; }
    else if (src == 3) { s.tol = 0.0; s.rel_tol = d.inner_rel_tol; s.max_iter = d.inner_max_iter; }
    else { s.tol = tol; s.rel_tol = rel_tol; s.max_iter = max_iter; }
}

// case c of the batch -> ks_gather[c][.] of the first case (one D2H copy)
__global__ void k_gather_ks(Batch bt)
{
    CASE_OF(bt);
    if (K.raw != 0) return;
    int c = 0;
    while (c + 1 < bt.n && (int)blockIdx.x >= bt.start[c + 1]) ++c;
    const int words = (int)(kNumKs * sizeof(KState) / sizeof(unsigned long long));
    const unsigned long long *src = reinterpret_cast<const unsigned long long *>(d.ks);
    unsigned long long *dst = reinterpret_cast<unsigned long long *>(bt.dc[0]->ks_gather + (size_t)c * kNumKs);
    for (int w = threadIdx.x; w < words; w += kBlock) dst[w] = src[w];
}

// ---- BiCG --------------------------------------------------------------

// p = z + beta p, p~ = z~ + beta p~ (z = r/diag, z~ = r~/diag)
template <class T>
__global__ void k_bicg_dir(Batch bt)
{
    CASE_OF(bt);
    const int i = K.raw * kBlock + threadIdx.x;
    if (i >= d.N) return;
    const BiArr<T> v = bi_arrays<T>(d);
    const long N = d.N;
    const T dg = v.diag[i];
    for (int c = 0; c < 3; ++c) {
        const KState &s = v.ks[c];
        if (s.done) continue;
        const long j = c * N + i;
        const T z = v.r[j] / dg, zt = v.rt[j] / dg;
        if (s.first) {
            v.p[j] = z;
            v.pt[j] = zt;
        } else {
            const T be = (T)s.beta;
            v.p[j] = z + be * v.p[j];
            v.pt[j] = zt + be * v.pt[j];
        }
    }
}

// q = A p, q~ = A^T p~, p~.q -> alpha
template <class T>
__global__ void __launch_bounds__(kBlock) k_bicg_spmv(Batch bt)
{
    CASE_OF(bt);
    const BiArr<T> v = bi_arrays<T>(d);
    int act[3];
    for (int c = 0; c < 3; ++c) act[c] = !v.ks[c].done;
    if (!act[0] && !act[1] && !act[2]) return;
    const Range rg = block_range(d.N, K);
    const long N = d.N;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int i = rg.beg + threadIdx.x; i < rg.end; i += kBlock) {
        for (int c = 0; c < 3; ++c) {
            if (!act[c]) continue;
            const T *p = v.p + c * N, *pt = v.pt + c * N;
            const T q = row_apply<T>(d, i, v.diag, v.up, v.lo, p);
            const T qt = row_apply<T>(d, i, v.diag, v.lo, v.up, pt);
            v.q[c * N + i] = q;
            v.qt[c * N + i] = qt;
            acc[c] += (double)pt[i] * (double)q;
        }
    }
    __shared__ double tot[3];
    if (reduce_last<3>(acc, d, K, tot) && threadIdx.x == 0) {
        for (int c = 0; c < 3; ++c) {
            if (!act[c]) continue;
            KState &s = v.ks[c];
            if (tot[c] == 0.0 || !isfinite(tot[c])) { set_done(s, FVM_ENUMERIC); s.iters += 1; }
            else s.alpha = s.rho / tot[c];
        }
    }
}

// x += alpha p, r -= alpha q, r~ -= alpha q~; rho = z.r~, |r| -> stop test, beta
template <class T>
__global__ void __launch_bounds__(kBlock) k_bicg_update(Batch bt)
{
    CASE_OF(bt);
    const BiArr<T> v = bi_arrays<T>(d);
    int act[3];
    T al[3];
    for (int c = 0; c < 3; ++c) { act[c] = !v.ks[c].done; al[c] = (T)v.ks[c].alpha; }
    if (!act[0] && !act[1] && !act[2]) return;
    const Range rg = block_range(d.N, K);
    const long N = d.N;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int i = rg.beg + threadIdx.x; i < rg.end; i += kBlock) {
        const T dg = v.diag[i];
        for (int c = 0; c < 3; ++c) {
            if (!act[c]) continue;
            const long j = c * N + i;
            v.x[j] += al[c] * v.p[j];
            const T r = v.r[j] - al[c] * v.q[j];
            const T rt = v.rt[j] - al[c] * v.qt[j];
            v.r[j] = r;
            v.rt[j] = rt;
            acc[c] += (double)(r / dg) * (double)rt;
            acc[3 + c] += fabs((double)r);
        }
    }
    __shared__ double tot[6];
    if (reduce_last<6>(acc, d, K, tot) && threadIdx.x == 0) {
        for (int c = 0; c < 3; ++c) {
            if (!act[c]) continue;
            KState &s = v.ks[c];
            s.iters += 1;
            s.nres = tot[3 + c] / s.nf;
            s.first = 0;
            if (!isfinite(s.nres)) set_done(s, FVM_ENUMERIC);
            else if (s.nres <= s.tol_eff) set_done(s, FVM_OK);
            else if (s.iters >= s.max_iter) set_done(s, FVM_WARN_MAXITER);
            else if (tot[c] == 0.0 || !isfinite(tot[c])) { set_done(s, FVM_ENUMERIC); s.iters += 1; }
            else {
                s.beta = tot[c] / s.rho;
                s.rho = tot[c];
            }
        }
    }
}

// FP64 start: sum x_c -> xbar_c
__global__ void __launch_bounds__(kBlock) k_bicg_sumx(Batch bt)
{
    CASE_OF(bt);
    const Range r = block_range(d.N, K);
    const long N = d.N;
    double v[3] = {0.0, 0.0, 0.0};
    for (int i = r.beg + threadIdx.x; i < r.end; i += kBlock)
        for (int c = 0; c < 3; ++c) v[c] += d.U[c * N + i];
    __shared__ double tot[3];
    if (reduce_last<3>(v, d, K, tot) && threadIdx.x == 0)
        for (int c = 0; c < 3; ++c) d.ks[c].xbar = tot[c] / (double)N;
}

// FP64 start: r = b - A x, r~ = r, normalisation, first rho = z.r~
// momentum solve start: r = b - A x, r~ = r; normalisation; rho = z.r~
// (BiCG) or r.r~ (BiCGStab, stab != 0)
__global__ void __launch_bounds__(kBlock) k_bicg_init(Batch bt, int stab)
{
    CASE_OF(bt);
    const Range rg = block_range(d.N, K);
    const long N = d.N;
    double xb[3];
    for (int c = 0; c < 3; ++c) xb[c] = d.ks[c].xbar;
    double v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};   // nf_c, |r|_c, rho_c
    for (int i = rg.beg + threadIdx.x; i < rg.end; i += kBlock) {
        const double a1 = row_sum(d, i, d.mdiag, d.upper, d.lower);
        const double dg = d.mdiag[i];
        for (int c = 0; c < 3; ++c) {
            const double *x = d.U + c * N;
            const double ax = row_apply<double>(d, i, d.mdiag, d.upper, d.lower, x);
            const double b = d.rhs[c * N + i];
            const double r = b - ax;
            d.r[c * N + i] = r;
            d.rt[c * N + i] = r;
            v[c] += fabs(ax - xb[c] * a1) + fabs(b - xb[c] * a1);
            v[3 + c] += fabs(r);
            v[6 + c] += stab ? r * r : (r / dg) * r;
        }
    }
    __shared__ double tot[9];
    if (reduce_last<9>(v, d, K, tot) && threadIdx.x == 0) {
        for (int c = 0; c < 3; ++c) {
            KState &s = d.ks[c];
            s.nf = tot[c] + 1e-20;
            s.nres0 = tot[3 + c] / s.nf;
            s.nres = s.nres0;
            s.tol_eff = fmax(s.tol, s.rel_tol * s.nres0);
            s.iters = 0;
            s.done = 0;
            s.status = FVM_OK;
            s.first = 1;
            s.beta = 0.0;
            s.omega = 1.0;
            s.half = 0;
            if (!isfinite(s.nres0)) set_done(s, FVM_ENUMERIC);
            else if (s.nres0 <= s.tol_eff) set_done(s, FVM_OK);
            else if (tot[6 + c] == 0.0 || !isfinite(tot[6 + c])) { set_done(s, FVM_ENUMERIC); s.iters = 1; }
            else s.rho = tot[6 + c];
        }
    }
}

// ---- BiCGStab (Barrett et al., Jacobi; three components) ----------------
// vectors: r, r~ = rt, p = pp, v = q, s = pt, t = qt, p^ = ph, s^ = sh

// p = r (first iteration) or r + beta (p - omega v); p^ = p / diag
__global__ void k_bs_dir(Batch bt)
{
    CASE_OF(bt);
    const int i = K.raw * kBlock + threadIdx.x;
    if (i >= d.N) return;
    const long N = d.N;
    const double dg = d.mdiag[i];
    for (int c = 0; c < 3; ++c) {
        const KState &s = d.ks[c];
        if (s.done) continue;
        const long j = c * N + i;
        const double p = s.first ? d.r[j] : d.r[j] + s.beta * (d.pp[j] - s.omega * d.q[j]);
        d.pp[j] = p;
        d.ph[j] = p / dg;
    }
}

// v = A p^; r~.v -> alpha = rho / (r~.v)
__global__ void __launch_bounds__(kBlock) k_bs_spmv_v(Batch bt)
{
    CASE_OF(bt);
    int act[3];
    for (int c = 0; c < 3; ++c) act[c] = !d.ks[c].done;
    if (!act[0] && !act[1] && !act[2]) return;
    const Range rg = block_range(d.N, K);
    const long N = d.N;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int i = rg.beg + threadIdx.x; i < rg.end; i += kBlock)
        for (int c = 0; c < 3; ++c) {
            if (!act[c]) continue;
            const double v = row_apply<double>(d, i, d.mdiag, d.upper, d.lower, d.ph + c * N);
            d.q[c * N + i] = v;
            acc[c] += d.rt[c * N + i] * v;
        }
    __shared__ double tot[3];
    if (reduce_last<3>(acc, d, K, tot) && threadIdx.x == 0)
        for (int c = 0; c < 3; ++c) {
            if (!act[c]) continue;
            KState &s = d.ks[c];
            if (tot[c] == 0.0 || !isfinite(tot[c])) { set_done(s, FVM_ENUMERIC); s.iters += 1; }
            else s.alpha = s.rho / tot[c];
        }
}

// s = r - alpha v, s^ = s / diag; |s| -> the half-step stopping test
__global__ void __launch_bounds__(kBlock) k_bs_s(Batch bt)
{
    CASE_OF(bt);
    int act[3];
    double al[3];
    for (int c = 0; c < 3; ++c) { act[c] = !d.ks[c].done; al[c] = d.ks[c].alpha; }
    if (!act[0] && !act[1] && !act[2]) return;
    const Range rg = block_range(d.N, K);
    const long N = d.N;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int i = rg.beg + threadIdx.x; i < rg.end; i += kBlock) {
        const double dg = d.mdiag[i];
        for (int c = 0; c < 3; ++c) {
            if (!act[c]) continue;
            const long j = c * N + i;
            const double sv = d.r[j] - al[c] * d.q[j];
            d.pt[j] = sv;
            d.sh[j] = sv / dg;
            acc[c] += fabs(sv);
        }
    }
    __shared__ double tot[3];
    if (reduce_last<3>(acc, d, K, tot) && threadIdx.x == 0)
        for (int c = 0; c < 3; ++c) {
            if (!act[c]) continue;
            KState &s = d.ks[c];
            s.iters += 1;
            const double ns = tot[c] / s.nf;
            if (!isfinite(ns)) { s.nres = ns; set_done(s, FVM_ENUMERIC); }
            else if (ns <= s.tol_eff) { s.nres = ns; s.half = 1; }
        }
}

// t = A s^; t.t and t.s -> omega (not for a system stopped at the half step)
__global__ void __launch_bounds__(kBlock) k_bs_spmv_t(Batch bt)
{
    CASE_OF(bt);
    int act[3];
    for (int c = 0; c < 3; ++c) act[c] = !d.ks[c].done && !d.ks[c].half;
    if (!act[0] && !act[1] && !act[2]) return;
    const Range rg = block_range(d.N, K);
    const long N = d.N;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int i = rg.beg + threadIdx.x; i < rg.end; i += kBlock)
        for (int c = 0; c < 3; ++c) {
            if (!act[c]) continue;
            const double t = row_apply<double>(d, i, d.mdiag, d.upper, d.lower, d.sh + c * N);
            d.qt[c * N + i] = t;
            acc[c] += t * t;
            acc[3 + c] += t * d.pt[c * N + i];
        }
    __shared__ double tot[6];
    if (reduce_last<6>(acc, d, K, tot) && threadIdx.x == 0)
        for (int c = 0; c < 3; ++c) {
            if (!act[c]) continue;
            KState &s = d.ks[c];
            if (tot[c] == 0.0 || !isfinite(tot[c]) || !isfinite(tot[3 + c])) set_done(s, FVM_ENUMERIC);
            else s.omega = tot[3 + c] / tot[c];
        }
}

// half step: x += alpha p^, r = s, stop; else x += alpha p^ + omega s^,
// r = s - omega t; |r| -> stop test; rho = r~.r, beta for the next step
__global__ void __launch_bounds__(kBlock) k_bs_update(Batch bt)
{
    CASE_OF(bt);
    int act[3], half[3];
    double al[3], om[3];
    for (int c = 0; c < 3; ++c) {
        act[c] = !d.ks[c].done;
        half[c] = d.ks[c].half;
        al[c] = d.ks[c].alpha;
        om[c] = d.ks[c].omega;
    }
    if (!act[0] && !act[1] && !act[2]) return;
    const Range rg = block_range(d.N, K);
    const long N = d.N;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int i = rg.beg + threadIdx.x; i < rg.end; i += kBlock)
        for (int c = 0; c < 3; ++c) {
            if (!act[c]) continue;
            const long j = c * N + i;
            if (half[c]) {
                d.U[j] += al[c] * d.ph[j];
                d.r[j] = d.pt[j];
            } else {
                d.U[j] += al[c] * d.ph[j] + om[c] * d.sh[j];
                const double r = d.pt[j] - om[c] * d.qt[j];
                d.r[j] = r;
                acc[c] += fabs(r);
                acc[3 + c] += d.rt[j] * r;
            }
        }
    __shared__ double tot[6];
    if (reduce_last<6>(acc, d, K, tot) && threadIdx.x == 0)
        for (int c = 0; c < 3; ++c) {
            if (!act[c]) continue;
            KState &s = d.ks[c];
            s.first = 0;
            if (half[c]) { s.half = 0; set_done(s, FVM_OK); continue; }
            s.nres = tot[c] / s.nf;
            if (!isfinite(s.nres)) set_done(s, FVM_ENUMERIC);
            else if (s.nres <= s.tol_eff) set_done(s, FVM_OK);
            else if (s.omega == 0.0) set_done(s, FVM_ENUMERIC);
            else if (s.iters >= s.max_iter) set_done(s, FVM_WARN_MAXITER);
            else if (tot[3 + c] == 0.0 || !isfinite(tot[3 + c])) { set_done(s, FVM_ENUMERIC); s.iters += 1; }
            else {
                s.beta = (tot[3 + c] / s.rho) * (s.alpha / s.omega);
                s.rho = tot[3 + c];
            }
        }
}

// ---- CG ----------------------------------------------------------------

// Streaming kernels take U cells per thread (grid SZ_CELL2 / SZ_CELL4): all
// loads of a thread are issued before the first use, so every wave keeps U
// times more bytes in flight than with one cell per thread.

// p = z + beta p (Jacobi z = r/diag; DIC z from the sweeps)
template <class T, int U>
__global__ void __launch_bounds__(kBlock) k_cg_dir(Batch bt, int dic, int rev)
{
    CASE_OF_DIR(bt, rev);
    const CGArr<T> v = cg_arrays<T>(d, dic);
    const KState &s = *v.ks;
    if (s.done) return;
    const bool first = s.first;
    const T beta = (T)s.beta;
    const Range rg = block_range(d.N, K);
    auto *__restrict__ p = gmem(v.p);
    const auto *__restrict__ z = gmem(v.z);
    const auto *__restrict__ r = gmem(v.r);
    const auto *__restrict__ dg = gmem(v.diag);
    for (int base = rg.beg; base < rg.end; base += U * kBlock) {
        T zv[U], pv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = base + u * kBlock + threadIdx.x;
            if (i < rg.end) {
                zv[u] = v.z ? (T)z[i] : r[i] / dg[i];
                pv[u] = first ? (T)0 : p[i];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = base + u * kBlock + threadIdx.x;
            if (i < rg.end) p[i] = first ? zv[u] : zv[u] + beta * pv[u];
        }
    }
}

// Pressure matrix values into the sliced-ELL copy (start of every pressure
// solve): FP64 cases fill sell_val, mixed cases the FP32 f_sell_val.  The
// pressure matrix is symmetric: both sides of a face take poff.
__global__ void __launch_bounds__(kBlock) k_sell_fill(Batch bt)
{
    CASE_OF(bt);
    const Range rg = block_range(d.N, K);
    if (rg.beg >= rg.end) return;
    const size_t base = (size_t)(rg.beg / kBlock) * d.sell_W * kBlock + threadIdx.x;
    for (int k = 0; k < d.sell_W; ++k) {
        const size_t e = base + (size_t)k * kBlock;
        const int fe = d.sell_fe[e];
        const double a = fe < 0 ? 0.0 : d.poff[fe >> 1];
        if (d.f_sell_val) d.f_sell_val[e] = (float)a;
        else d.sell_val[e] = a;
    }
}

// q = A p, p.q -> alpha, on the sliced-ELL copy: one block = one slice of
// 256 consecutive cells, one cell per thread; slot k of the slice is one
// coalesced stream of coefficients, and in a regular slice the gathered
// p[i + off_k] are consecutive too.  Padding entries hold 0 (their column
// is clamped into the mesh).  The cell sums its entries in ascending
// column order after the diagonal term.
//
// FP32 (mixed precision) uses the difference form
//   (A32 p)_i = sum_k a_k p_j + (exc_i - sum_k a_k) p_i,
// exc_i being the FP64 row sum rounded once.  Rounding the diagonal and the
// off-diagonals to FP32 separately would perturb every row sum by
// O(eps32 diag): on a pressure system whose only non-zero row sums are a few
// boundary or reference cells that moves the smallest eigenvalues by O(1)
// and stalls CG.  In difference form the FP32 operator is the graph
// Laplacian of the rounded face weights plus the rounded row sums,
// spectrally within (1 +- eps32) of the FP64 one.  Products of FP32 values
// are exact in FP64 and the sums are FP64.  In a slice of mode 2 (no
// fixed-pressure face, no reference pin) every row sum is exactly zero, and
// the FP64 value is only the rounding residue of forming it: exc_i = 0 there,
// and it is not read.
// the sliced-ELL structure a product reads, held in registers by a kernel
// that loops over slices (the case descriptor lives in memory the product's
// stores could alias, so its fields would otherwise be reloaded per slice)
struct SellView {
    const int32_t *mode, *off, *mir, *col;
    int N, W;
};
__device__ __forceinline__ SellView sell_view(const DevCase &d)
{
    return SellView{d.sell_mode, d.sell_off, d.sell_mir, d.sell_col, d.N, d.sell_W};
}

// one row of the product: q_i (not stored) and p_i q_i
template <class T>
struct Row {
    T q;
    double pq;
};
template <class T, int WC>
__device__ __forceinline__ Row<T> spmv_row(const SellView &sw, const CGArr<T> &v, int sl, int i)
{
    // per-slice tables are read as uniform scalar loads, coefficients and
    // gathers as global-space vector loads (no flat-load waits)
    typedef const __attribute__((address_space(4))) int cint;
    typedef const __attribute__((address_space(1))) T gT;
    typedef const __attribute__((address_space(1))) int gint;
    constexpr bool kDiff = sizeof(T) == 4;
    const int W = WC > 0 ? WC : sw.W;
    const size_t base = (size_t)sl * W * kBlock + (i & (kBlock - 1));   // slices start at multiples of kBlock
    gT *__restrict__ sv = (gT *)v.sval;
    gT *__restrict__ val = sv + base;
    gT *__restrict__ p = (gT *)v.p;
    const double pi = (double)p[i];
    const int mode = ((cint *)sw.mode)[sl];
    double qa, so = 0.0;
    if (WC > 0 && mode != 1) {
        // regular slice, slot count known: the slice's offsets and mirror
        // slots are fetched together, then every load is issued before use.
        // Mode 2 (FP64): the diagonal is minus the row's coefficient sum,
        // formed in the order the pressure assembly forms it (upper entries
        // by ascending column, then lower ones), so it equals the stored
        // diagonal bit for bit and is not read.
        cint *off = (cint *)(sw.off + (size_t)sl * W);
        cint *mir = (cint *)(sw.mir + (size_t)sl * W);
        const int last = sw.N - 1;
        T a[WC > 0 ? WC : 1], pj[WC > 0 ? WC : 1];
        int o[WC > 0 ? WC : 1], m[WC > 0 ? WC : 1];
#pragma unroll
        for (int k = 0; k < W; ++k) {
            o[k] = off[k];
            m[k] = mir[k];
        }
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const int j = min(max(i + o[k], 0), last);
            // a lower slot with a mirror reads a_ji from the neighbour's
            // upper slot (a stream read moments ago, still in cache) instead
            // of its own copy of the same value
            gT *src = m[k] < 0 ? val + (size_t)k * kBlock
                               : sv + ((size_t)(j / kBlock) * W + m[k]) * kBlock + (j % kBlock);
            a[k] = *src;
            pj[k] = p[j];
        }
        if (kDiff) qa = 0.0;
        else if (mode == 2) {
            double dg = 0.0;
#pragma unroll
            for (int k = 0; k < W; ++k)
                if (o[k] > 0) dg += -(double)a[k];
#pragma unroll
            for (int k = 0; k < W; ++k)
                if (o[k] < 0) dg += -(double)a[k];
            qa = dg * pi;
        } else qa = (double)((gT *)v.diag)[i] * pi;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            qa += (double)a[k] * (double)pj[k];
            if (kDiff) so += (double)a[k];
        }
    } else {
        qa = kDiff ? 0.0 : (double)((gT *)v.diag)[i] * pi;
        if (mode != 1) {
            cint *off = (cint *)(sw.off + (size_t)sl * W);
            cint *mir = (cint *)(sw.mir + (size_t)sl * W);
            const int last = sw.N - 1;
#pragma unroll 6
            for (int k = 0; k < W; ++k) {
                const int j = min(max(i + off[k], 0), last);
                const int mk = mir[k];
                gT *src = mk < 0 ? val + (size_t)k * kBlock : sv + ((size_t)(j / kBlock) * W + mk) * kBlock + (j % kBlock);
                const T a = *src;
                qa += (double)a * (double)p[j];
                if (kDiff) so += (double)a;
            }
        } else {
            gint *__restrict__ col = (gint *)(sw.col + base);
#pragma unroll 6
            for (int k = 0; k < W; ++k) {
                const T a = val[(size_t)k * kBlock];
                qa += (double)a * (double)p[col[(size_t)k * kBlock]];
                if (kDiff) so += (double)a;
            }
        }
    }
    const double exc = kDiff && mode != 2 ? (double)((gT *)v.exc)[i] : 0.0;
    const T q = kDiff ? (T)(qa + (exc - so) * pi) : (T)qa;
    return Row<T>{q, pi * (double)q};
}

template <class T, int WC>
__device__ __forceinline__ double spmv_cell(const SellView &sw, const CGArr<T> &v, int sl, int i)
{
    const Row<T> r = spmv_row<T, WC>(sw, v, sl, i);
    v.q[i] = r.q;
    return r.pq;
}

template <class T, int WC>
__device__ __forceinline__ double spmv_cell(const DevCase &d, const CGArr<T> &v, int sl, int i)
{
    return spmv_cell<T, WC>(sell_view(d), v, sl, i);
}

// A block takes the slices of its range one after the other (one cell per
// thread per slice), so its set-up (case descriptor, controls) and the grid
// reduction at its end are paid once for several slices.  WC > 0: the slot
// count is fixed at compile time (6 on hex meshes): the loop is unrolled and
// a slice's offsets and mirror slots are fetched together.
template <class T, int WC>
__global__ void __launch_bounds__(kBlock) k_cg_spmv(Batch bt, int dic, int rev)
{
    CASE_OF_DIR(bt, rev);
    const CGArr<T> v = cg_arrays<T>(d, dic);
    if (v.ks->done) return;
    const Range rg = block_range(d.N, K);
    const SellView sw = sell_view(d);
    double acc[1] = {0.0};
    for (int base = rg.beg; base < rg.end; base += kBlock) {
        const int i = base + threadIdx.x;
        if (i < rg.end) acc[0] += spmv_cell<T, WC>(sw, v, base / kBlock, i);
    }
    __shared__ double tot[1];
    if (reduce_last<1>(acc, d, K, tot) && threadIdx.x == 0) {
        KState &s = *v.ks;
        if (!(tot[0] > 0.0) || !isfinite(tot[0])) { set_done(s, FVM_ENUMERIC); s.iters += 1; }
        else s.alpha = s.rho / tot[0];
    }
}

// G consecutive cells (i0 a multiple of G) of a 7-point regular slice per
// thread: slots (-c, -b, -1, +1, +b, +c) with b and c multiples of G, the
// three lower slots mirrored from the upper ones (5, 4, 3 for 0, 1, 2), and
// every neighbour of the slice inside the mesh (the interior slices of a
// lexicographic hex box).  Own slots, p, the diagonal, q and the neighbour
// groups at offsets +-b and +-c move as single 16-byte accesses; the -1
// neighbour of the first cell and the +1 neighbour of the last one are
// single elements, the other +-1 neighbours are the group's own values.
// Each cell's sum is formed exactly as spmv_cell forms it.
template <class T, int G>
struct Grp {
    T e[G];
};
// G elements at a multiple of G, as one vector load
template <class T, int G>
__device__ __forceinline__ Grp<T, G> ld_grp(const __attribute__((address_space(1))) T *a)
{
    typedef T V __attribute__((ext_vector_type(G)));
    const V w = *(const __attribute__((address_space(1))) V *)a;
    Grp<T, G> r;
#pragma unroll
    for (int g = 0; g < G; ++g) r.e[g] = w[g];
    return r;
}

// whether slice sl has the 7-point form above (uniform over the slice)
template <int G>
__device__ __forceinline__ bool slice_7pt(const SellView &sw, int sl)
{
    typedef const __attribute__((address_space(4))) int cint;
    cint *op = (cint *)(sw.off + (size_t)sl * 6);
    cint *mp = (cint *)(sw.mir + (size_t)sl * 6);
    // every entry is loaded, then the tests are combined without branches
    int o[6], m[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        o[k] = op[k];
        m[k] = mp[k];
    }
    const int c = o[5], b = o[4];
    return (o[2] == -1) & (o[3] == 1) & (o[1] == -b) & (o[0] == -c) & (b > 1) & (c > b) & (((b | c) & (G - 1)) == 0) &
           (m[0] == 5) & (m[1] == 4) & (m[2] == 3) & (m[3] < 0) & (m[4] < 0) & (m[5] < 0) &
           (sl * kBlock - c >= 0) & (sl * kBlock + kBlock - 1 + c <= sw.N - 1);
}

template <class T, int G>
__device__ __forceinline__ double spmv_group(const SellView &sw, const CGArr<T> &v, int sl, int i0, int mode)
{
    typedef const __attribute__((address_space(4))) int cint;
    typedef const __attribute__((address_space(1))) T gT;
    constexpr int W = 6;
    constexpr bool kDiff = sizeof(T) == 4;
    gT *__restrict__ sv = (gT *)v.sval;
    gT *__restrict__ val = sv + (size_t)sl * W * kBlock + (i0 & (kBlock - 1));
    gT *__restrict__ p = (gT *)v.p;
    cint *off = (cint *)(sw.off + (size_t)sl * W);
    const int c = off[5], b = off[4];
    // loads, all issued before the first use
    const Grp<T, G> pp = ld_grp<T, G>(p + i0);
    const Grp<T, G> o3 = ld_grp<T, G>(val + 3 * kBlock), o4 = ld_grp<T, G>(val + 4 * kBlock),
                    o5 = ld_grp<T, G>(val + 5 * kBlock);
    const int jc = i0 - c, jb = i0 - b, j1 = i0 - 1;
    const Grp<T, G> m0 = ld_grp<T, G>(sv + ((size_t)(jc / kBlock) * W + 5) * kBlock + (jc & (kBlock - 1)));
    const Grp<T, G> m1 = ld_grp<T, G>(sv + ((size_t)(jb / kBlock) * W + 4) * kBlock + (jb & (kBlock - 1)));
    const T m2 = sv[((size_t)(j1 / kBlock) * W + 3) * kBlock + (j1 & (kBlock - 1))];
    const Grp<T, G> xc = ld_grp<T, G>(p + jc), xb = ld_grp<T, G>(p + jb), yb = ld_grp<T, G>(p + i0 + b),
                    yc = ld_grp<T, G>(p + i0 + c);
    const T xm = p[j1], yp = p[i0 + G];
    Grp<T, G> dg{}, ex{};
    if (!kDiff && mode != 2) dg = ld_grp<T, G>((gT *)v.diag + i0);
    if (kDiff && mode != 2) ex = ld_grp<T, G>((gT *)v.exc + i0);
    // slot k: coefficient and neighbour value of cell i0 + g
    T a[G][W], x[G][W];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        a[g][0] = m0.e[g];
        a[g][1] = m1.e[g];
        a[g][2] = g == 0 ? m2 : o3.e[g > 0 ? g - 1 : 0];
        a[g][3] = o3.e[g];
        a[g][4] = o4.e[g];
        a[g][5] = o5.e[g];
        x[g][0] = xc.e[g];
        x[g][1] = xb.e[g];
        x[g][2] = g == 0 ? xm : pp.e[g > 0 ? g - 1 : 0];
        x[g][3] = g == G - 1 ? yp : pp.e[g < G - 1 ? g + 1 : 0];
        x[g][4] = yb.e[g];
        x[g][5] = yc.e[g];
    }
    double q[G], so[G];
#pragma unroll
    for (int g = 0; g < G; ++g) {
        so[g] = 0.0;
        if (kDiff) q[g] = 0.0;
        else if (mode == 2) {
            // upper slots (3, 4, 5), then lower ones (0, 1, 2)
            double d = 0.0;
#pragma unroll
            for (int k = 3; k < W; ++k) d += -(double)a[g][k];
#pragma unroll
            for (int k = 0; k < 3; ++k) d += -(double)a[g][k];
            q[g] = d * (double)pp.e[g];
        } else q[g] = (double)dg.e[g] * (double)pp.e[g];
    }
#pragma unroll
    for (int k = 0; k < W; ++k)
#pragma unroll
        for (int g = 0; g < G; ++g) {
            q[g] += (double)a[g][k] * (double)x[g][k];
            if (kDiff) so[g] += (double)a[g][k];
        }
    typedef T V __attribute__((ext_vector_type(G)));
    V w;
    double part = 0.0;
#pragma unroll
    for (int g = 0; g < G; ++g) {
        const double pi = (double)pp.e[g];
        const T r = kDiff ? (T)(q[g] + ((mode != 2 ? (double)ex.e[g] : 0.0) - so[g]) * pi) : (T)q[g];
        w[g] = r;
        part += pi * (double)r;
    }
    *(__attribute__((address_space(1))) V *)(v.q + i0) = w;
    return part;
}

// q = A p on slot count 6 with G cells per thread (16-byte groups): the
// block's threads split into G parts, each taking every G-th slice of the
// block's range; slices not of the 7-point form (explicit, partial,
// boundary planes, other stencils) go cell by cell.  A case with fewer than
// half of its slices of that form (random or RCM numbering, small boxes)
// runs one cell per thread throughout (G cells of a thread would be G
// lanes apart in its fallback).  FP64 takes pairs; the
// FP32 product stays one cell per thread (groups of 2 or 4 floats measured
// 3% and 12% slower: more registers per cell, fewer resident waves).
template <class T, int G>
__global__ void __launch_bounds__(kBlock) k_cg_spmv_grp(Batch bt, int dic, int rev)
{
    typedef const __attribute__((address_space(4))) int cint;
    CASE_OF_DIR(bt, rev);
    const CGArr<T> v = cg_arrays<T>(d, dic);
    if (v.ks->done) return;
    const Range rg = block_range(d.N, K);
    const SellView sw = sell_view(d);
    double acc[1] = {0.0};
    if (2L * d.sell_n7 < (d.N + kBlock - 1) / kBlock) {
        // most slices are not of the 7-point form: one cell per thread, as
        // in k_cg_spmv (the choice is the case's own, so a case computes the
        // same bits alone and in any batch)
        for (int base = rg.beg; base < rg.end; base += kBlock) {
            const int i = base + threadIdx.x;
            if (i < rg.end) acc[0] += spmv_cell<T, 6>(sw, v, base / kBlock, i);
        }
    } else if (rg.beg < rg.end) {
        constexpr int per = kBlock / G;   // threads per slice (whole waves)
        const int sl_end = (rg.end + kBlock - 1) / kBlock;
        const int u0 = G * (threadIdx.x & (per - 1));
        const int sub = __builtin_amdgcn_readfirstlane((int)(threadIdx.x / per));
        for (int sl = rg.beg / kBlock + sub; sl < sl_end; sl += G) {
            const int i0 = sl * kBlock + u0;
            const int mode = ((cint *)sw.mode)[sl];
            if (mode != 1 && (sl + 1) * kBlock <= rg.end && slice_7pt<G>(sw, sl))
                acc[0] += spmv_group<T, G>(sw, v, sl, i0, mode);
            else {
#pragma unroll
                for (int g = 0; g < G; ++g)
                    if (i0 + g < rg.end) acc[0] += spmv_cell<T, 6>(sw, v, sl, i0 + g);
            }
        }
    }
    __shared__ double tot[1];
    if (reduce_last<1>(acc, d, K, tot) && threadIdx.x == 0) {
        KState &s = *v.ks;
        if (!(tot[0] > 0.0) || !isfinite(tot[0])) { set_done(s, FVM_ENUMERIC); s.iters += 1; }
        else s.alpha = s.rho / tot[0];
    }
}

// FP64: x += alpha p, r -= alpha q, |r| -> stop test; Jacobi: rho, beta
template <int U>
__global__ void __launch_bounds__(kBlock) k_cg_update(Batch bt, int dic, int rev)
{
    CASE_OF_DIR(bt, rev);
    const CGArr<double> v = cg_arrays<double>(d, dic);
    if (v.ks->done) return;
    const double al = v.ks->alpha;
    const Range rg = block_range(d.N, K);
    double acc[2] = {0.0, 0.0};
    auto *__restrict__ x = gmem(v.x);
    auto *__restrict__ rr = gmem(v.r);
    const auto *__restrict__ p = gmem((const double *)v.p);
    const auto *__restrict__ q = gmem((const double *)v.q);
    const auto *__restrict__ dg = gmem(v.diag);
    for (int base = rg.beg; base < rg.end; base += U * kBlock) {
        double xv[U], rv[U], pv[U], qv[U], dv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = base + u * kBlock + threadIdx.x;
            if (i < rg.end) {
                xv[u] = x[i]; rv[u] = rr[i]; pv[u] = p[i]; qv[u] = q[i];
                dv[u] = dic ? 1.0 : dg[i];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = base + u * kBlock + threadIdx.x;
            if (i < rg.end) {
                x[i] = xv[u] + al * pv[u];
                const double r = rv[u] - al * qv[u];
                rr[i] = r;
                acc[0] += fabs(r);
                if (!dic) acc[1] += r * (r / dv[u]);
            }
        }
    }
    __shared__ double tot[2];
    if (reduce_last<2>(acc, d, K, tot) && threadIdx.x == 0) {
        KState &s = *v.ks;
        s.iters += 1;
        s.nres = tot[0] / s.nf;
        s.first = 0;
        if (!isfinite(s.nres)) set_done(s, FVM_ENUMERIC);
        else if (s.nres <= s.tol_eff) set_done(s, FVM_OK);
        else if (s.iters >= s.max_iter) set_done(s, FVM_WARN_MAXITER);
        else if (!dic) {
            if (!(tot[1] > 0.0) || !isfinite(tot[1])) { set_done(s, FVM_ENUMERIC); s.iters += 1; }
            else {
                s.beta = tot[1] / s.rho;
                s.rho = tot[1];
            }
        }
    }
}

__global__ void __launch_bounds__(kBlock) k_pcg_sumx(Batch bt)
{
    CASE_OF(bt);
    const Range r = block_range(d.N, K);
    double v[1] = {0.0};
    for (int i = r.beg + threadIdx.x; i < r.end; i += kBlock) v[0] += d.p[i];
    __shared__ double tot[1];
    if (reduce_last<1>(v, d, K, tot) && threadIdx.x == 0) d.ks[3].xbar = tot[0] / (double)d.N;
}

// FP64 start: r = b - A x; normalisation; Jacobi: first rho = r.(r/diag)
// dic: 0 Jacobi, 1 DIC, 2 AMG (the last two compute z and rho themselves)
__global__ void __launch_bounds__(kBlock) k_pcg_init(Batch bt, int dic)
{
    CASE_OF(bt);
    const Range rg = block_range(d.N, K);
    const double xb = d.ks[3].xbar;
    double v[3] = {0.0, 0.0, 0.0};
    for (int i = rg.beg + threadIdx.x; i < rg.end; i += kBlock) {
        const double a1 = row_sum(d, i, d.pdiag, d.poff, d.poff);
        const double ax = row_apply<double>(d, i, d.pdiag, d.poff, d.poff, d.p);
        const double b = d.pb[i];
        const double r = b - ax;
        d.r[i] = r;
        v[0] += fabs(ax - xb * a1) + fabs(b - xb * a1);
        v[1] += fabs(r);
        if (!dic) v[2] += r * (r / d.pdiag[i]);
        else if (dic == 1) {
            clear_word(d.dq, i);
            clear_word(d.yq, i);
            clear_word(d.zq, i);
        }
    }
    __shared__ double tot[3];
    if (reduce_last<3>(v, d, K, tot) && threadIdx.x == 0) {
        KState &s = d.ks[3];
        s.nf = tot[0] + 1e-20;
        s.nres0 = tot[1] / s.nf;
        s.nres = s.nres0;
        s.tol_eff = fmax(s.tol, s.rel_tol * s.nres0);
        s.iters = 0;
        s.done = 0;
        s.status = FVM_OK;
        s.first = 1;
        s.beta = 0.0;
        if (!isfinite(s.nres0)) set_done(s, FVM_ENUMERIC);
        else if (s.nres0 <= s.tol_eff) set_done(s, FVM_OK);
        else if (!dic) {
            if (!(tot[2] > 0.0) || !isfinite(tot[2])) { set_done(s, FVM_ENUMERIC); s.iters = 1; }
            else s.rho = tot[2];
        }
    }
}

// ---------------------------------------------------------------------------
// DIC triangular sweeps, sync-free in level order, on one XCD
//
// The diagonal-only incomplete Cholesky factor D* and the two triangular
// solves of M = (D* + L) D*^-1 (D* + U) are recurrences over the lower
// (upper) neighbours of each cell.  Cells are processed in the order of the
// dependency levels computed at mesh ingest, in tiles of 256 cells claimed
// through an atomic ticket, so every dependency of a tile lies in a tile
// that has already been claimed by a running block.
//
// A sweep is a chain of as many dependent steps as there are levels, so its
// time is set by the latency of handing a value from one CU to another.  The
// sweep therefore runs on a single XCD: the first block of the launch elects
// its XCD, blocks on the other XCDs leave at once, and the elected XCD's
// blocks stay resident and claim tiles until none are left.  A value is
// published with a plain 64-bit store into an array pre-filled with a NaN
// sentinel; it lands in the XCD's L2, where device-scope loads from the same
// XCD see it (about half the latency of a store written through to memory).
// The value is its own ready flag, so no fence is needed and a reader polls
// exactly the word it consumes.  Polling is bounded: past the limit the
// value is published as NaN, which the solver reports as a breakdown instead
// of hanging.  Per cell the sums run over neighbours in ascending index.
// ---------------------------------------------------------------------------

// device-scope load of a published word
__device__ __forceinline__ unsigned long long dic_ld(const double *a, int j) { return gld(a + j); }

__device__ __forceinline__ bool dic_try(const double *a, int j, double &v)
{
    const unsigned long long b = dic_ld(a, j);
    if (b == kSentinel) return false;
    v = __longlong_as_double((long long)b);
    return true;
}

// plain (XCD-local) 64-bit store of a published value
__device__ __forceinline__ void dic_put(double *a, int i, double v)
{
    unsigned long long b = (unsigned long long)__double_as_longlong(v);
    if (b == kSentinel) b = kQNaN;
    __hip_atomic_store((gword *)(a + i), b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// the NaN sentinel through a global-space store
__device__ __forceinline__ void clear_slot(double *a, long i) { *(gword *)(a + i) = kSentinel; }

// hardware XCD (XCC) id of the executing wave
__device__ __forceinline__ unsigned int xcc_id() { return __builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 15u; }

// MODE 0: D*_i = A_ii - sum_{j<i} a_ij^2 / D*_j
// MODE 1: y_i = (r_i - sum_{j<i} a_ij y_j) / D*_i      (also clears z)
// MODE 2: z_i = y_i - (sum_{j>i} a_ij z_j) / D*_i      (reverse order; r.z)
//
// A cell's dependency list (neighbour index and coefficient) is read into
// registers before polling, so each poll round is one batch of independent
// device-scope loads of the values still missing; once all are present the
// sum is formed in ascending neighbour order.  D register slots (4 for hex
// meshes, else 8; fewer registers keep more waves resident); meshes whose
// cells have more than D dependencies take a streaming path that consumes
// them one at a time.

// Blocks claim tiles of 256 consecutive entries of the level order (reversed
// for MODE 2); each wave of the block takes 64 of them.  Before its lanes
// poll, a wave waits on a single word: the value at the position dic_lag
// places before its first one (dic_lag is at least twice the widest level,
// and at least 8192).  Only the waves within that distance of the
// completion front poll their dependencies; the ones further ahead poll one
// address, which keeps the XCD's L2 free for the hand-over traffic at the
// front.  Positions complete in roughly increasing order and the gate lies
// before the wave's own positions, so the earliest unfinished position is
// never gated: the sweep always progresses.
constexpr int kChunk = 64;

// DIC coefficients in level order, refilled at the start of every solve
// (the pressure matrix is symmetric: both triangles read poff)
__global__ void __launch_bounds__(kBlock) k_dic_fill(Batch bt)
{
    CASE_OF(bt);
    const Range rg = block_range(d.N, K);
    const long N = d.N;
    for (int q = rg.beg + threadIdx.x; q < rg.end; q += kBlock) {
        for (int k = 0; k < d.dW_lo; ++k) {
            const int f = d.dl_face[k * N + q];
            d.dl_val[k * N + q] = f >= 0 ? d.poff[f] : 0.0;
        }
        for (int k = 0; k < d.dW_hi; ++k) {
            const int f = d.du_face[k * N + q];
            d.du_val[k * N + q] = f >= 0 ? d.poff[f] : 0.0;
        }
    }
}

// One wave processes 64 consecutive positions of the processing order (the
// level order, reversed for MODE 2).  Dependencies, their coefficients and
// the published values are all indexed by level position, so a lane's loads
// are coalesced slot streams and a level's inputs form one contiguous range.
template <int MODE, int D>
__device__ __forceinline__ double dic_chunk(const DevCase &d, int chunk)
{
    const int n = d.N;
    const long N = n;
    const int lane = threadIdx.x & 63;
    const int q = chunk * kChunk + lane;          // processing position
    const bool live = q < n;
    const int fq = live ? (MODE == 2 ? n - 1 - q : q) : 0;   // level position
    const int i = live ? gmem(d.lvl_cells)[fq] : 0;
    const int W = MODE == 2 ? d.dW_hi : d.dW_lo;
    const auto *__restrict__ DP = gmem(MODE == 2 ? (const int *)d.du_pos : (const int *)d.dl_pos);
    const auto *__restrict__ DV = gmem(MODE == 2 ? (const double *)d.du_val : (const double *)d.dl_val);
    double *const src = MODE == 0 ? d.dq : (MODE == 1 ? d.yq : d.zq);
    // everything the publication needs is read from the case descriptor
    // now: the descriptor lives in memory that the stores below could
    // alias, so a field read after them would be a load between a value
    // becoming ready and its publication
    double *const dq = d.dq, *const yq = d.yq, *const zq = d.zq;
    auto *const dstar = gmem(d.dstar);
    auto *const zout = gmem(d.z);
    unsigned int *const ticket = d.ticket;
    // all slots are loaded at once (independent loads); a cell's
    // dependencies fill slots 0..nd-1
    const bool fast = W <= D;
    int js[D];
    double as[D], vs[D];
#pragma unroll
    for (int t = 0; t < D; ++t) {
        js[t] = -1; as[t] = 0.0; vs[t] = 0.0;
        if (live && fast && t < W) {
            js[t] = DP[t * N + fq];
            as[t] = DV[t * N + fq];
        }
    }
    int nd = 0;
    if (fast) {
#pragma unroll
        for (int t = 0; t < D; ++t) nd += js[t] >= 0 ? 1 : 0;
    } else if (live) {
        while (nd < W && DP[nd * N + fq] >= 0) ++nd;
    }
    // the cell's own inputs (the diagonal or r, D*_i, y_i; r_i for r.z),
    // produced by earlier launches, are read before any wait
    double acc = 0.0;
    if (live && MODE != 2) acc = MODE == 0 ? gmem(d.pdiag)[i] : gmem(d.r)[i];
    const double dsi = (MODE != 0 && live) ? gmem(dq)[fq] : 1.0;
    const double yi = (MODE == 2 && live) ? gmem(yq)[fq] : 0.0;
    const double ri = (MODE == 2 && live) ? gmem(d.r)[i] : 0.0;
    // a wave whose lanes all depend only on positions inside the chunk (or on
    // nothing) has no reason to wait; the test is a max over the wave's lanes
    // (this form schedules better than a ballot).  Waves of the streaming
    // path are not gated.
    int gate = -1;   // processing position of the latest dependency before this chunk
#pragma unroll
    for (int t = 0; t < D; ++t) {
        if (js[t] >= 0) {
            const int pd = MODE == 2 ? n - 1 - js[t] : js[t];
            if (pd < chunk * kChunk && pd > gate) gate = pd;
        }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) gate = max(gate, __shfl_xor(gate, o, 64));
    const int gq = chunk * kChunk - d.dic_lag;   // the gate, in processing order
    if (gate >= 0 && gq >= 0) {
        // every lane loads the same word: one request per wave; the wait
        // is long (the gate lies about two levels behind the wave's first
        // position), so the wave sleeps ~2000 cycles between polls and
        // leaves the issue slots and the L2 to the waves at the front
        const int gp = MODE == 2 ? n - 1 - gq : gq;
        double v;
        for (int sp = 0; sp < kSpinLimit && !dic_try(src, gp, v); ++sp) __builtin_amdgcn_s_sleep(32);
    }
    // past the gate the wave is near the completion front: it takes issue
    // priority over the waves still waiting at their gates
    __builtin_amdgcn_s_setprio(2);
    unsigned int missing = fast ? (nd >= 32 ? 0xffffffffu : ((1u << nd) - 1u)) : 0u;
    int k = 0;                // streaming path cursor
    double part = 0.0;
    bool fin = !live;
    int spins = 0;
    // the loop exits only when the whole wave is done: work placed on a
    // divergent loop-exit path would run after every lane has left the loop,
    // holding back values that other lanes of the wave wait for
    for (;;) {
        if (!fin) {
            bool ready;
            if (fast) {
                // issue every dependency load of the lane before the first
                // comparison, so that they overlap instead of each waiting
                // for the previous one
                unsigned long long bv[D];
#pragma unroll
                for (int t = 0; t < D; ++t) bv[t] = t < nd ? dic_ld(src, js[t]) : 0ull;
#pragma unroll
                for (int t = 0; t < D; ++t)
                    if (((missing >> t) & 1u) && bv[t] != kSentinel) {
                        vs[t] = __longlong_as_double((long long)bv[t]);
                        missing &= ~(1u << t);
                    }
                ready = missing == 0u;
                if (ready) {
#pragma unroll
                    for (int t = 0; t < D; ++t) {
                        if (t < nd) {
                            if (MODE == 0) acc -= as[t] * as[t] / vs[t];
                            else if (MODE == 1) acc -= as[t] * vs[t];
                            else acc += as[t] * vs[t];
                        }
                    }
                }
            } else {
                ready = true;
                while (k < nd) {
                    double v;
                    if (!dic_try(src, DP[k * N + fq], v)) { ready = false; break; }
                    const double a = DV[k * N + fq];
                    if (MODE == 0) acc -= a * a / v;
                    else if (MODE == 1) acc -= a * v;
                    else acc += a * v;
                    ++k;
                }
            }
            if (ready) {
                if (MODE == 0) { dic_put(dq, fq, acc); dstar[i] = acc; }
                else if (MODE == 1) { dic_put(yq, fq, acc / dsi); clear_slot(zq, fq); }
                else {
                    const double zi = yi - acc / dsi;
                    dic_put(zq, fq, zi);
                    zout[i] = zi;
                    clear_slot(yq, fq);
                    part = ri * zi;
                }
                fin = true;
            } else if (++spins > kSpinLimit) {
                dic_put(src, fq, __longlong_as_double((long long)kQNaN));
                if (MODE == 0) dstar[i] = __longlong_as_double((long long)kQNaN);
                if (MODE == 2) {
                    zout[i] = __longlong_as_double((long long)kQNaN);
                    part = __longlong_as_double((long long)kQNaN);
                }
                ticket[8] = 1u;
                fin = true;
            }
        }
        if (__all(fin)) break;
        __builtin_amdgcn_s_sleep(1);
    }
    __builtin_amdgcn_s_setprio(0);
    return part;
}

template <int MODE, int D>
__global__ void __launch_bounds__(kBlock, D == 4 ? 6 : 4) k_dic_sweep(Batch bt)
{
    CASE_OF(bt);
    if (d.ks[3].done) return;
    __shared__ int s_on, s_tile;
    if (threadIdx.x == 0) {
        // elect the XCD of the first block to arrive (ticket[5] = xcc + 1)
        const unsigned int x = xcc_id() + 1u;
        unsigned int e = 0u;
        __hip_atomic_compare_exchange_strong(&d.ticket[5], &e, x, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        s_on = e == 0u || e == x;
    }
    __syncthreads();
    double part = 0.0;
    if (s_on) {
        // the block claims tiles until none are left; the waves of a tile
        // work on consecutive cells (shared cache lines)
        for (;;) {
            if (threadIdx.x == 0) s_tile = (int)atomicAdd(&d.ticket[1], 1u);
            __syncthreads();
            const int tile = s_tile;
            __syncthreads();
            if ((long)tile * kBlock >= d.N) break;
            part += dic_chunk<MODE, D>(d, tile * kWaves + (threadIdx.x >> 6));
        }
    }
    if (MODE == 2) {
        double v[1] = {part};
        __shared__ double tot[1];
        if (reduce_last<1>(v, d, K, tot) && threadIdx.x == 0) {
            KState &s = d.ks[3];
            __hip_atomic_store(&d.ticket[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            __hip_atomic_store(&d.ticket[5], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (!(tot[0] > 0.0) || !isfinite(tot[0])) { set_done(s, FVM_ENUMERIC); s.iters += 1; }
            else if (s.iters == 0) s.rho = tot[0];
            else {
                s.beta = tot[0] / s.rho;
                s.rho = tot[0];
            }
        }
    } else {
        __syncthreads();
        if (threadIdx.x == 0) {
            const unsigned int t = __hip_atomic_fetch_add(&d.ticket[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (t == (unsigned int)K.G - 1) {
                __hip_atomic_store(&d.ticket[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&d.ticket[2], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&d.ticket[5], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

__global__ void k_dic_reset(Batch bt)
{
    CASE_OF(bt);
    const int i = K.raw * kBlock + threadIdx.x;
    if (i == 0) {
        d.ks[3].done = 0;
        d.ks[3].iters = 0;
        d.ks[3].status = FVM_OK;
    }
    if (i >= d.N) return;
    clear_word(d.dq, i);
    clear_word(d.yq, i);
    clear_word(d.zq, i);
}

// ---------------------------------------------------------------------------
// Mixed precision
//
// Pressure (CG): the FP32 recurrence runs uninterrupted (FP32 matrix in
// difference form, r, p, q; FP64 sums and dots) while the solution is
// accumulated in FP64 (x += alpha p); whenever the recurrence residual has
// fallen 10x since the last replacement it is replaced by the true FP64
// residual b - A x, and convergence is decided on that true residual: when
// the recurrence residual reaches the tolerance (or the iteration limit is
// reached) the iteration pauses (done = 2) until the next replacement
// (launched after every few iterations) checks it.
// Restarting an FP32 CG from each refined residual instead would throw its
// Krylov space away, which on these pressure systems multiplies the
// iteration count several times over.
//
// Momentum (BiCG, a few iterations per solve): FP64 iterative refinement
// around FP32 BiCG solves of A e = s r to a relative reduction eta
// (s = N / sum|r| keeps the demoted residual O(1)), x += e / s.
// States: ks[0..3] the FP64 solves, ks[4..6] the FP32 momentum inner solves.
// ---------------------------------------------------------------------------

// FP32 copies of the assembled matrix values (the topology is shared)
__global__ void k_mx_cvt(Batch bt, int kind)
{
    CASE_OF(bt);
    const int t = K.raw * kBlock + threadIdx.x;
    if (kind == 1) {
        if (t < d.N) {
            d.f_pdiag[t] = (float)d.pdiag[t];
            d.f_pexc[t] = (float)row_sum(d, t, d.pdiag, d.poff, d.poff);
        }
        if (t < d.Fi) d.f_poff[t] = (float)d.poff[t];
    } else {
        if (t < d.N) d.f_diag[t] = (float)d.mdiag[t];
        if (t < d.Fi) { d.f_up[t] = (float)d.upper[t]; d.f_lo[t] = (float)d.lower[t]; }
    }
}

// ---- pressure: FP32 recurrence, FP64 solution ---------------------------

// start: r32 = r64 (from the FP64 start kernel), rho = r32.(r32/diag32)
__global__ void __launch_bounds__(kBlock) k_rr_start(Batch bt)
{
    CASE_OF(bt);
    if (d.ks[3].done) return;
    const Range rg = block_range(d.N, K);
    double acc[1] = {0.0};
    for (int i = rg.beg + threadIdx.x; i < rg.end; i += kBlock) {
        const float r = (float)d.r[i];
        d.f_r[i] = r;
        acc[0] += (double)r * (double)(r / d.f_pdiag[i]);
    }
    __shared__ double tot[1];
    if (reduce_last<1>(acc, d, K, tot) && threadIdx.x == 0) {
        KState &s = d.ks[3];
        s.scale = s.nres;     // recurrence residual at the last replacement
        if (!(tot[0] > 0.0) || !isfinite(tot[0])) { set_done(s, FVM_ENUMERIC); s.iters = 1; }
        else s.rho = tot[0];
    }
}

// x64 += alpha p32, r32 -= alpha q32; |r32| and rho (FP64 accumulation).
// The solution stays FP64: an FP32 solution increment would carry rounding
// noise of relative size eps32, which A amplifies by up to its condition
// number in the true residual.
template <int U>
__global__ void __launch_bounds__(kBlock) k_rr_update(Batch bt, int rev)
{
    CASE_OF_DIR(bt, rev);
    if (d.ks[3].done) return;
    const double al = d.ks[3].alpha;
    const float alf = (float)al;
    const Range rg = block_range(d.N, K);
    double acc[2] = {0.0, 0.0};
    auto *__restrict__ x = gmem(d.p);
    const auto *__restrict__ p = gmem((const float *)d.f_p);
    const auto *__restrict__ q = gmem((const float *)d.f_q);
    const auto *__restrict__ dg = gmem((const float *)d.f_pdiag);
    auto *__restrict__ r = gmem(d.f_r);
    for (int base = rg.beg; base < rg.end; base += U * kBlock) {
        double xv[U];
        float pv[U], qv[U], rv[U], dv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = base + u * kBlock + threadIdx.x;
            if (i < rg.end) { xv[u] = x[i]; pv[u] = p[i]; qv[u] = q[i]; rv[u] = r[i]; dv[u] = dg[i]; }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = base + u * kBlock + threadIdx.x;
            if (i < rg.end) {
                x[i] = xv[u] + al * (double)pv[u];
                const float ri = rv[u] - alf * qv[u];
                r[i] = ri;
                acc[0] += fabs((double)ri);
                acc[1] += (double)ri * (double)(ri / dv[u]);
            }
        }
    }
    __shared__ double tot[2];
    if (reduce_last<2>(acc, d, K, tot) && threadIdx.x == 0) {
        KState &s = d.ks[3];
        s.iters += 1;
        s.nres = tot[0] / s.nf;
        s.first = 0;
        s.xbar = s.rho;   // rho of the previous iteration (for a replacement)
        if (!isfinite(s.nres)) set_done(s, FVM_ENUMERIC);
        else if (s.nres <= s.tol_eff || s.iters >= s.max_iter) s.done = 2;   // verify on the true residual
        else if (!(tot[1] > 0.0) || !isfinite(tot[1])) { set_done(s, FVM_ENUMERIC); s.iters += 1; }
        else {
            s.beta = tot[1] / s.rho;
            s.rho = tot[1];
        }
    }
}

// residual replacement: r64 = b - A64 x64; r32 = r64; taken when the
// iteration is paused or the recurrence residual fell 10x since the last
// replacement; rho and beta continue from the true residual
__global__ void __launch_bounds__(kBlock) k_rr_replace(Batch bt)
{
    CASE_OF(bt);
    const KState &s0 = d.ks[3];
    if (s0.done == 1) return;
    if (s0.done == 0 && !(s0.nres < 0.1 * s0.scale)) return;
    const Range rg = block_range(d.N, K);
    double acc[2] = {0.0, 0.0};
    for (int i = rg.beg + threadIdx.x; i < rg.end; i += kBlock) {
        const double r = d.pb[i] - row_apply<double>(d, i, d.pdiag, d.poff, d.poff, d.p);
        const float rf = (float)r;
        d.f_r[i] = rf;
        acc[0] += fabs(r);
        acc[1] += (double)rf * (double)(rf / d.f_pdiag[i]);
    }
    __shared__ double tot[2];
    if (reduce_last<2>(acc, d, K, tot) && threadIdx.x == 0) {
        KState &s = d.ks[3];
        const double nres = tot[0] / s.nf;
        s.nres = nres;
        s.scale = nres;
        if (!isfinite(nres)) set_done(s, FVM_ENUMERIC);
        else if (nres <= s.tol_eff) set_done(s, FVM_OK);
        else if (s.iters >= s.max_iter) set_done(s, FVM_WARN_MAXITER);
        else if (!(tot[1] > 0.0) || !isfinite(tot[1])) { set_done(s, FVM_ENUMERIC); s.iters += 1; }
        else {
            s.beta = s.first ? 0.0 : tot[1] / s.xbar;
            s.rho = tot[1];
            s.done = 0;
        }
    }
}

// FP32 pressure update step of the recurrence: p = z + beta p is k_cg_dir<float>;
// q = A32 p is k_cg_spmv<float>

// ---- momentum: FP64 refinement around restarted FP32 BiCG ----------------

__device__ __forceinline__ double mx_scale(const KState &o, int N) { return (double)N / (o.nres * o.nf); }

// inner start: r_in = s r (FP32), e = 0, inner normalisation sum|r_in|,
// rho = (r_in/diag).r_in
__global__ void __launch_bounds__(kBlock) k_mx_inner_init(Batch bt)
{
    CASE_OF(bt);
    int act[3];
    double sc[3];
    for (int c = 0; c < 3; ++c) {
        act[c] = !d.ks[c].done;
        sc[c] = act[c] ? mx_scale(d.ks[c], d.N) : 0.0;
    }
    if (!act[0] && !act[1] && !act[2]) {
        if (K.raw == 0 && threadIdx.x == 0)
            for (int c = 0; c < 3; ++c) { set_done(d.ks[4 + c], FVM_OK); d.ks[4 + c].iters = 0; }
        return;
    }
    const Range rg = block_range(d.N, K);
    const long N = d.N;
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int i = rg.beg + threadIdx.x; i < rg.end; i += kBlock) {
        const float dg = d.f_diag[i];
        for (int c = 0; c < 3; ++c) {
            if (!act[c]) continue;
            const long j = c * N + i;
            const float r = (float)(sc[c] * d.r[j]);
            d.f_r[j] = r;
            d.f_rt[j] = r;
            d.f_x[j] = 0.0f;
            v[c] += fabs((double)r);
            v[3 + c] += (double)(r / dg) * (double)r;
        }
    }
    __shared__ double tot[6];
    if (reduce_last<6>(v, d, K, tot) && threadIdx.x == 0) {
        for (int c = 0; c < 3; ++c) {
            KState &s = d.ks[4 + c];
            if (!act[c]) { set_done(s, FVM_OK); s.iters = 0; continue; }
            s.nf = tot[c];
            s.nres0 = 1.0;
            s.nres = 1.0;
            s.tol_eff = fmax(s.tol, s.rel_tol);
            s.iters = 0;
            s.done = 0;
            s.status = FVM_OK;
            s.first = 1;
            s.beta = 0.0;
            if (!isfinite(tot[c]) || !(tot[c] > 0.0)) set_done(s, FVM_ENUMERIC);
            else if (tot[3 + c] == 0.0 || !isfinite(tot[3 + c])) { set_done(s, FVM_ENUMERIC); s.iters = 1; }
            else s.rho = tot[3 + c];
        }
    }
}

// x += e / s (FP64), for the components whose outer loop is still running
// and whose inner solve did not break down (its e is then discarded)
__global__ void k_mx_correct(Batch bt)
{
    CASE_OF(bt);
    const int i = K.raw * kBlock + threadIdx.x;
    if (i >= d.N) return;
    for (int c = 0; c < 3; ++c) {
        const KState &o = d.ks[c];
        if (o.done || d.ks[4 + c].status == FVM_ENUMERIC) continue;
        const double s = mx_scale(o, d.N);
        const long j = (long)c * d.N + i;
        d.U[j] += (double)d.f_x[j] / s;
    }
}

// outer residual after a correction: r = b - A x (FP64), nres, stop test;
// the inner iterations are added to the outer count
__global__ void __launch_bounds__(kBlock) k_mx_resid(Batch bt)
{
    CASE_OF(bt);
    int act[3];
    for (int c = 0; c < 3; ++c) act[c] = !d.ks[c].done;
    if (!act[0] && !act[1] && !act[2]) return;
    const Range rg = block_range(d.N, K);
    const long N = d.N;
    double v[3] = {0, 0, 0};
    for (int i = rg.beg + threadIdx.x; i < rg.end; i += kBlock) {
        for (int c = 0; c < 3; ++c) {
            if (!act[c]) continue;
            const long j = c * N + i;
            const double r = d.rhs[j] - row_apply<double>(d, i, d.mdiag, d.upper, d.lower, d.U + c * N);
            d.r[j] = r;
            v[c] += fabs(r);
        }
    }
    __shared__ double tot[3];
    if (reduce_last<3>(v, d, K, tot) && threadIdx.x == 0) {
        for (int c = 0; c < 3; ++c) {
            if (!act[c]) continue;
            KState &o = d.ks[c];
            const KState &in = d.ks[4 + c];
            o.iters += in.iters;
            o.nres = tot[c] / o.nf;
            if (!isfinite(o.nres)) set_done(o, FVM_ENUMERIC);
            else if (in.status == FVM_ENUMERIC) set_done(o, kStatusFallback);
            else if (o.nres <= o.tol_eff) set_done(o, FVM_OK);
            else if (o.iters >= o.max_iter) set_done(o, FVM_WARN_MAXITER);
        }
    }
}

// FP64 BiCG restart of the components marked kStatusFallback, from the
// current iterate: r (already b - A x) is its own shadow, rho = z.r~
__global__ void __launch_bounds__(kBlock) k_bicg_fallback(Batch bt)
{
    CASE_OF(bt);
    int act[3];
    for (int c = 0; c < 3; ++c) act[c] = d.ks[c].status == kStatusFallback;
    if (!act[0] && !act[1] && !act[2]) return;
    const Range rg = block_range(d.N, K);
    const long N = d.N;
    double v[3] = {0.0, 0.0, 0.0};
    for (int i = rg.beg + threadIdx.x; i < rg.end; i += kBlock) {
        const double dg = d.mdiag[i];
        for (int c = 0; c < 3; ++c) {
            if (!act[c]) continue;
            const long j = c * N + i;
            const double r = d.r[j];
            d.rt[j] = r;
            v[c] += (r / dg) * r;
        }
    }
    __shared__ double tot[3];
    if (reduce_last<3>(v, d, K, tot) && threadIdx.x == 0) {
        for (int c = 0; c < 3; ++c) {
            if (!act[c]) continue;
            KState &s = d.ks[c];
            s.first = 1;
            s.beta = 0.0;
            s.status = FVM_OK;
            s.done = 0;
            if (tot[c] == 0.0 || !isfinite(tot[c])) { set_done(s, FVM_ENUMERIC); s.iters += 1; }
            else s.rho = tot[c];
        }
    }
}

// ---------------------------------------------------------------------------
// Whole PISO steps of small cases, one workgroup per case
//
// A case of a few thousand cells cannot fill the GPU, and at that size a
// solve driven by a few launches per Krylov iteration is bound by launch and
// host-polling latency.  k_solo_piso runs complete PISO steps of a case in
// one workgroup of kSolo threads: the same per-cell and per-face arithmetic
// as the launched kernels (the el_* functions and the same Krylov
// recurrences), phases separated by workgroup barriers, sums formed in LDS
// in a fixed order, and the Krylov loops on the device: every thread sees
// the same totals and the same stopping decisions.  A launch holds many
// cases side by side, one per CU.  The case's Krylov states live in LDS
// during the step; at the end the last step's record is left in the case's
// state slots for the host: ks[0..2] momentum, ks[3..6] the pressure solves,
// ks[7] a summary (iters: pressure solves of the last step, status: worst
// status over the steps, done: steps completed, first: 1 when a step failed
// and was rolled back).  Scope (the host checks it): orthogonal meshes, at
// most 4 pressure correctors without non-orthogonal correction, Jacobi CG
// and BiCG, FP64 or mixed precision.
// ---------------------------------------------------------------------------
constexpr int kSolo = 512;
constexpr int kSoloWaves = kSolo / 64;

struct SoloShared {
    double red[12][kSoloWaves];
    KState ks[kNumKs];
    KState rec[kNumKs];
};

#define SOLO_FOR(var, n) for (int var = (int)threadIdx.x; var < (n); var += kSolo)

// fixed-order workgroup sum of NV values; every thread receives the totals
template <int NV>
__device__ __forceinline__ void solo_sum(double (&v)[NV], SoloShared &sh)
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    wave_sum(v);
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) sh.red[k][wv] = v[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        double t = sh.red[k][0];
        for (int w = 1; w < kSoloWaves; ++w) t += sh.red[k][w];
        v[k] = t;
    }
}

// the controls of k_set_ctl (src 0 momentum, 1 pressure, 3 FP32 inner)
__device__ __forceinline__ void solo_ctl(const DevCase &d, KState &s, int src)
{
    if (src == 0) { s.tol = d.u_tol; s.rel_tol = d.u_rel_tol; s.max_iter = d.u_max_iter; }
    else if (src == 1) { s.tol = d.p_tol; s.rel_tol = d.p_rel_tol; s.max_iter = d.p_max_iter; }
    else { s.tol = 0.0; s.rel_tol = d.inner_rel_tol; s.max_iter = d.inner_max_iter; }
}

// ---- momentum: BiCG on the three components (k_bicg_* in one workgroup)

// FP64 start (k_bicg_sumx, k_bicg_init): r = b - A x, r~ = r, n_f, rho
__device__ void solo_bicg_init(const DevCase &d, SoloShared &sh)
{
    const long N = d.N;
    double xb[3] = {0.0, 0.0, 0.0};
    SOLO_FOR(i, d.N) for (int c = 0; c < 3; ++c) xb[c] += d.U[c * N + i];
    solo_sum<3>(xb, sh);
    for (int c = 0; c < 3; ++c) xb[c] /= (double)N;
    double v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    SOLO_FOR(i, d.N) {
        const double a1 = row_sum(d, i, d.mdiag, d.upper, d.lower);
        const double dg = d.mdiag[i];
        for (int c = 0; c < 3; ++c) {
            const double ax = row_apply<double>(d, i, d.mdiag, d.upper, d.lower, d.U + c * N);
            const double b = d.rhs[c * N + i];
            const double r = b - ax;
            d.r[c * N + i] = r;
            d.rt[c * N + i] = r;
            v[c] += fabs(ax - xb[c] * a1) + fabs(b - xb[c] * a1);
            v[3 + c] += fabs(r);
            v[6 + c] += (r / dg) * r;
        }
    }
    solo_sum<9>(v, sh);
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; ++c) {
            KState &s = sh.ks[c];
            s.xbar = xb[c];
            s.nf = v[c] + 1e-20;
            s.nres0 = v[3 + c] / s.nf;
            s.nres = s.nres0;
            s.tol_eff = fmax(s.tol, s.rel_tol * s.nres0);
            s.iters = 0;
            s.done = 0;
            s.status = FVM_OK;
            s.first = 1;
            s.beta = 0.0;
            if (!isfinite(s.nres0)) set_done(s, FVM_ENUMERIC);
            else if (s.nres0 <= s.tol_eff) set_done(s, FVM_OK);
            else if (v[6 + c] == 0.0 || !isfinite(v[6 + c])) { set_done(s, FVM_ENUMERIC); s.iters = 1; }
            else s.rho = v[6 + c];
        }
    __syncthreads();
}

// BiCG iterations until the three systems (states ks0..ks0+2) are done;
// at most `limit` iterations (the launched solver's bound)
template <class T>
__device__ void solo_bicg_iterate(const DevCase &d, SoloShared &sh, const BiArr<T> &v, int ks0, long limit)
{
    const long N = d.N;
    KState *ks = sh.ks + ks0;
    for (long it = 0; it < limit; ++it) {
        int act[3];
        for (int c = 0; c < 3; ++c) act[c] = !ks[c].done;
        if (!act[0] && !act[1] && !act[2]) break;
        // direction (k_bicg_dir)
        SOLO_FOR(i, d.N) {
            const T dg = v.diag[i];
            for (int c = 0; c < 3; ++c) {
                if (!act[c]) continue;
                const long j = c * N + i;
                const T z = v.r[j] / dg, zt = v.rt[j] / dg;
                if (ks[c].first) {
                    v.p[j] = z;
                    v.pt[j] = zt;
                } else {
                    const T be = (T)ks[c].beta;
                    v.p[j] = z + be * v.p[j];
                    v.pt[j] = zt + be * v.pt[j];
                }
            }
        }
        __syncthreads();
        // products (k_bicg_spmv)
        double acc[3] = {0.0, 0.0, 0.0};
        SOLO_FOR(i, d.N) {
            for (int c = 0; c < 3; ++c) {
                if (!act[c]) continue;
                const T *p = v.p + c * N, *pt = v.pt + c * N;
                const T q = row_apply<T>(d, i, v.diag, v.up, v.lo, p);
                const T qt = row_apply<T>(d, i, v.diag, v.lo, v.up, pt);
                v.q[c * N + i] = q;
                v.qt[c * N + i] = qt;
                acc[c] += (double)pt[i] * (double)q;
            }
        }
        solo_sum<3>(acc, sh);
        if (threadIdx.x == 0)
            for (int c = 0; c < 3; ++c) {
                if (!act[c]) continue;
                KState &s = ks[c];
                if (acc[c] == 0.0 || !isfinite(acc[c])) { set_done(s, FVM_ENUMERIC); s.iters += 1; }
                else s.alpha = s.rho / acc[c];
            }
        __syncthreads();
        // update (k_bicg_update)
        T al[3];
        for (int c = 0; c < 3; ++c) { act[c] = !ks[c].done; al[c] = (T)ks[c].alpha; }
        double u6[6] = {0, 0, 0, 0, 0, 0};
        SOLO_FOR(i, d.N) {
            const T dg = v.diag[i];
            for (int c = 0; c < 3; ++c) {
                if (!act[c]) continue;
                const long j = c * N + i;
                v.x[j] += al[c] * v.p[j];
                const T r = v.r[j] - al[c] * v.q[j];
                const T rt = v.rt[j] - al[c] * v.qt[j];
                v.r[j] = r;
                v.rt[j] = rt;
                u6[c] += (double)(r / dg) * (double)rt;
                u6[3 + c] += fabs((double)r);
            }
        }
        solo_sum<6>(u6, sh);
        if (threadIdx.x == 0)
            for (int c = 0; c < 3; ++c) {
                if (!act[c]) continue;
                KState &s = ks[c];
                s.iters += 1;
                s.nres = u6[3 + c] / s.nf;
                s.first = 0;
                if (!isfinite(s.nres)) set_done(s, FVM_ENUMERIC);
                else if (s.nres <= s.tol_eff) set_done(s, FVM_OK);
                else if (s.iters >= s.max_iter) set_done(s, FVM_WARN_MAXITER);
                else if (u6[c] == 0.0 || !isfinite(u6[c])) { set_done(s, FVM_ENUMERIC); s.iters += 1; }
                else {
                    s.beta = u6[c] / s.rho;
                    s.rho = u6[c];
                }
            }
        __syncthreads();
    }
    // a bound reached without a stop flag: the launched driver reports an
    // error there too
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; ++c)
            if (!ks[c].done) set_done(ks[c], FVM_ENUMERIC);
    __syncthreads();
}

// momentum solve: FP64 BiCG, or FP64 refinement around restarted FP32 BiCG
__device__ void solo_momentum(const DevCase &d, SoloShared &sh, bool mixed)
{
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; ++c) solo_ctl(d, sh.ks[c], 0);
    __syncthreads();
    solo_bicg_init(d, sh);
    if (!mixed) {
        solo_bicg_iterate<double>(d, sh, bi_arrays<double>(d), 0, (long)d.u_max_iter + 1);
        return;
    }
    const long N = d.N;
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; ++c) solo_ctl(d, sh.ks[4 + c], 3);
    SOLO_FOR(t, d.N > d.Fi ? d.N : d.Fi) {   // k_mx_cvt, momentum
        if (t < d.N) d.f_diag[t] = (float)d.mdiag[t];
        if (t < d.Fi) { d.f_up[t] = (float)d.upper[t]; d.f_lo[t] = (float)d.lower[t]; }
    }
    __syncthreads();
    for (int outer = 0;; ++outer) {
        int act[3];
        for (int c = 0; c < 3; ++c) act[c] = !sh.ks[c].done;
        if (!act[0] && !act[1] && !act[2]) break;
        if (outer >= 1000) {
            if (threadIdx.x == 0)
                for (int c = 0; c < 3; ++c)
                    if (act[c]) set_done(sh.ks[c], FVM_ENUMERIC);
            __syncthreads();
            break;
        }
        // inner start (k_mx_inner_init)
        double sc[3];
        for (int c = 0; c < 3; ++c) sc[c] = act[c] ? mx_scale(sh.ks[c], d.N) : 0.0;
        double v[6] = {0, 0, 0, 0, 0, 0};
        SOLO_FOR(i, d.N) {
            const float dg = d.f_diag[i];
            for (int c = 0; c < 3; ++c) {
                if (!act[c]) continue;
                const long j = c * N + i;
                const float r = (float)(sc[c] * d.r[j]);
                d.f_r[j] = r;
                d.f_rt[j] = r;
                d.f_x[j] = 0.0f;
                v[c] += fabs((double)r);
                v[3 + c] += (double)(r / dg) * (double)r;
            }
        }
        solo_sum<6>(v, sh);
        if (threadIdx.x == 0)
            for (int c = 0; c < 3; ++c) {
                KState &s = sh.ks[4 + c];
                if (!act[c]) { set_done(s, FVM_OK); s.iters = 0; continue; }
                s.nf = v[c];
                s.nres0 = 1.0;
                s.nres = 1.0;
                s.tol_eff = fmax(s.tol, s.rel_tol);
                s.iters = 0;
                s.done = 0;
                s.status = FVM_OK;
                s.first = 1;
                s.beta = 0.0;
                if (!isfinite(v[c]) || !(v[c] > 0.0)) set_done(s, FVM_ENUMERIC);
                else if (v[3 + c] == 0.0 || !isfinite(v[3 + c])) { set_done(s, FVM_ENUMERIC); s.iters = 1; }
                else s.rho = v[3 + c];
            }
        __syncthreads();
        solo_bicg_iterate<float>(d, sh, bi_arrays<float>(d), 4, (long)d.inner_max_iter + 1);
        // correction and outer residual (k_mx_correct, k_mx_resid)
        int keep[3];
        for (int c = 0; c < 3; ++c) keep[c] = act[c] && sh.ks[4 + c].status != FVM_ENUMERIC;
        SOLO_FOR(i, d.N)
            for (int c = 0; c < 3; ++c)
                if (keep[c]) d.U[(long)c * N + i] += (double)d.f_x[(long)c * N + i] / sc[c];
        __syncthreads();
        double w[3] = {0, 0, 0};
        SOLO_FOR(i, d.N)
            for (int c = 0; c < 3; ++c) {
                if (!act[c]) continue;
                const long j = c * N + i;
                const double r = d.rhs[j] - row_apply<double>(d, i, d.mdiag, d.upper, d.lower, d.U + c * N);
                d.r[j] = r;
                w[c] += fabs(r);
            }
        solo_sum<3>(w, sh);
        if (threadIdx.x == 0)
            for (int c = 0; c < 3; ++c) {
                if (!act[c]) continue;
                KState &o = sh.ks[c];
                const KState &in = sh.ks[4 + c];
                o.iters += in.iters;
                o.nres = w[c] / o.nf;
                if (!isfinite(o.nres)) set_done(o, FVM_ENUMERIC);
                else if (in.status == FVM_ENUMERIC) set_done(o, kStatusFallback);
                else if (o.nres <= o.tol_eff) set_done(o, FVM_OK);
                else if (o.iters >= o.max_iter) set_done(o, FVM_WARN_MAXITER);
            }
        __syncthreads();
    }
    // components whose FP32 inner solve broke down continue in FP64
    // (k_bicg_fallback, then the FP64 BiCG iterations)
    int fb[3];
    for (int c = 0; c < 3; ++c) fb[c] = sh.ks[c].status == kStatusFallback;
    if (!fb[0] && !fb[1] && !fb[2]) return;
    double v[3] = {0.0, 0.0, 0.0};
    SOLO_FOR(i, d.N) {
        const double dg = d.mdiag[i];
        for (int c = 0; c < 3; ++c) {
            if (!fb[c]) continue;
            const long j = c * N + i;
            const double r = d.r[j];
            d.rt[j] = r;
            v[c] += (r / dg) * r;
        }
    }
    solo_sum<3>(v, sh);
    if (threadIdx.x == 0)
        for (int c = 0; c < 3; ++c) {
            if (!fb[c]) continue;
            KState &s = sh.ks[c];
            s.first = 1;
            s.beta = 0.0;
            s.status = FVM_OK;
            s.done = 0;
            if (v[c] == 0.0 || !isfinite(v[c])) { set_done(s, FVM_ENUMERIC); s.iters += 1; }
            else s.rho = v[c];
        }
    __syncthreads();
    solo_bicg_iterate<double>(d, sh, bi_arrays<double>(d), 0, (long)d.u_max_iter + 1);
}

// ---- pressure: Jacobi CG (k_cg_*, k_pcg_init; mixed: k_rr_*) -----------

template <class T>
__device__ __forceinline__ Row<T> solo_spmv_row(const DevCase &d, const CGArr<T> &v, int i)
{
    const SellView sw = sell_view(d);
    return d.sell_W == 6 ? spmv_row<T, 6>(sw, v, i / kBlock, i) : spmv_row<T, 0>(sw, v, i / kBlock, i);
}

// Cells per thread per round of the whole-step kernel's CG passes: a round
// issues the loads of all its cells before the first store (the arrays are
// not known to be distinct, so a store keeps later loads behind it, and one
// cell at a time would pay a memory round trip per cell).  A thread still
// takes cells i = tid, tid + kSolo, ... in that order, so the sums are
// formed as before.
constexpr int kSoloU = 4;

// one FP64 or FP32 CG iteration on state s (dir, product, update of the
// launched kernels); mixed: the FP32 recurrence with the FP64 solution
template <class T>
__device__ void solo_cg_iteration(const DevCase &d, SoloShared &sh, const CGArr<T> &v, KState &s)
{
    constexpr bool kMixed = sizeof(T) == 4;
    const bool first = s.first;
    const T beta = (T)s.beta;
    const int N = d.N;
    for (int b = (int)threadIdx.x; b < N; b += kSolo * kSoloU) {
        T rv[kSoloU], dv[kSoloU], pv[kSoloU];
#pragma unroll
        for (int u = 0; u < kSoloU; ++u) {
            const int i = b + u * kSolo;
            if (i < N) {
                rv[u] = v.r[i];
                dv[u] = v.diag[i];
                pv[u] = first ? (T)0 : v.p[i];
            }
        }
#pragma unroll
        for (int u = 0; u < kSoloU; ++u) {
            const int i = b + u * kSolo;
            if (i < N) {
                const T z = rv[u] / dv[u];
                v.p[i] = first ? z : z + beta * pv[u];
            }
        }
    }
    __syncthreads();
    double pq[1] = {0.0};
    for (int b = (int)threadIdx.x; b < N; b += kSolo * 2) {
        Row<T> rw[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int i = b + u * kSolo;
            if (i < N) rw[u] = solo_spmv_row<T>(d, v, i);
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            const int i = b + u * kSolo;
            if (i < N) {
                v.q[i] = rw[u].q;
                pq[0] += rw[u].pq;
            }
        }
    }
    solo_sum<1>(pq, sh);
    if (threadIdx.x == 0) {
        if (!(pq[0] > 0.0) || !isfinite(pq[0])) { set_done(s, FVM_ENUMERIC); s.iters += 1; }
        else s.alpha = s.rho / pq[0];
    }
    __syncthreads();
    if (s.done) return;
    const double al = s.alpha;
    double acc[2] = {0.0, 0.0};
    for (int b = (int)threadIdx.x; b < N; b += kSolo * kSoloU) {
        double xv[kSoloU];
        T pv[kSoloU], rv[kSoloU], qv[kSoloU], dv[kSoloU];
#pragma unroll
        for (int u = 0; u < kSoloU; ++u) {
            const int i = b + u * kSolo;
            if (i < N) {
                xv[u] = d.p[i];
                pv[u] = v.p[i];
                rv[u] = v.r[i];
                qv[u] = v.q[i];
                dv[u] = v.diag[i];
            }
        }
#pragma unroll
        for (int u = 0; u < kSoloU; ++u) {
            const int i = b + u * kSolo;
            if (i >= N) continue;
            d.p[i] = xv[u] + al * (double)pv[u];
            if (!kMixed) {
                const double r = (double)rv[u] - al * (double)qv[u];
                v.r[i] = (T)r;
                acc[0] += fabs(r);
                acc[1] += r * (r / (double)dv[u]);
            } else {
                const float ri = (float)rv[u] - (float)al * (float)qv[u];
                v.r[i] = (T)ri;
                acc[0] += fabs((double)ri);
                acc[1] += (double)ri * (double)(ri / (float)dv[u]);
            }
        }
    }
    solo_sum<2>(acc, sh);
    if (threadIdx.x == 0) {
        s.iters += 1;
        s.nres = acc[0] / s.nf;
        s.first = 0;
        if (kMixed) s.xbar = s.rho;   // rho of the previous iteration (for a replacement)
        if (!isfinite(s.nres)) set_done(s, FVM_ENUMERIC);
        else if (kMixed && (s.nres <= s.tol_eff || s.iters >= s.max_iter)) s.done = 2;   // verify on the true residual
        else if (!kMixed && s.nres <= s.tol_eff) set_done(s, FVM_OK);
        else if (!kMixed && s.iters >= s.max_iter) set_done(s, FVM_WARN_MAXITER);
        else if (!(acc[1] > 0.0) || !isfinite(acc[1])) { set_done(s, FVM_ENUMERIC); s.iters += 1; }
        else {
            s.beta = acc[1] / s.rho;
            s.rho = acc[1];
        }
    }
    __syncthreads();
}

// mixed precision: residual replacement (k_rr_replace)
__device__ void solo_rr_replace(const DevCase &d, SoloShared &sh, KState &s)
{
    if (s.done == 1) return;
    if (s.done == 0 && !(s.nres < 0.1 * s.scale)) return;
    double acc[2] = {0.0, 0.0};
    SOLO_FOR(i, d.N) {
        const double r = d.pb[i] - row_apply<double>(d, i, d.pdiag, d.poff, d.poff, d.p);
        const float rf = (float)r;
        d.f_r[i] = rf;
        acc[0] += fabs(r);
        acc[1] += (double)rf * (double)(rf / d.f_pdiag[i]);
    }
    solo_sum<2>(acc, sh);
    if (threadIdx.x == 0) {
        const double nres = acc[0] / s.nf;
        s.nres = nres;
        s.scale = nres;
        if (!isfinite(nres)) set_done(s, FVM_ENUMERIC);
        else if (nres <= s.tol_eff) set_done(s, FVM_OK);
        else if (s.iters >= s.max_iter) set_done(s, FVM_WARN_MAXITER);
        else if (!(acc[1] > 0.0) || !isfinite(acc[1])) { set_done(s, FVM_ENUMERIC); s.iters += 1; }
        else {
            s.beta = s.first ? 0.0 : acc[1] / s.xbar;
            s.rho = acc[1];
            s.done = 0;
        }
    }
    __syncthreads();
}

// pressure solve of the assembled system (pdiag, poff, pb), x = p
__device__ void solo_pressure(const DevCase &d, SoloShared &sh, bool mixed)
{
    KState &s = sh.ks[3];
    if (threadIdx.x == 0) solo_ctl(d, s, 1);
    // sliced-ELL values (k_sell_fill) and, mixed, the FP32 copies (k_mx_cvt)
    const int nsl = (d.N + kBlock - 1) / kBlock;
    SOLO_FOR(e, nsl * d.sell_W * kBlock) {
        const int fe = d.sell_fe[e];
        const double a = fe < 0 ? 0.0 : d.poff[fe >> 1];
        if (mixed) d.f_sell_val[e] = (float)a;
        else d.sell_val[e] = a;
    }
    if (mixed)
        SOLO_FOR(t, d.N > d.Fi ? d.N : d.Fi) {
            if (t < d.N) {
                d.f_pdiag[t] = (float)d.pdiag[t];
                d.f_pexc[t] = (float)row_sum(d, t, d.pdiag, d.poff, d.poff);
            }
            if (t < d.Fi) d.f_poff[t] = (float)d.poff[t];
        }
    // start (k_pcg_sumx, k_pcg_init with Jacobi)
    double xb[1] = {0.0};
    SOLO_FOR(i, d.N) xb[0] += d.p[i];
    solo_sum<1>(xb, sh);
    const double xbar = xb[0] / (double)d.N;
    double v[3] = {0.0, 0.0, 0.0};
    SOLO_FOR(i, d.N) {
        const double a1 = row_sum(d, i, d.pdiag, d.poff, d.poff);
        const double ax = row_apply<double>(d, i, d.pdiag, d.poff, d.poff, d.p);
        const double b = d.pb[i];
        const double r = b - ax;
        d.r[i] = r;
        v[0] += fabs(ax - xbar * a1) + fabs(b - xbar * a1);
        v[1] += fabs(r);
        v[2] += r * (r / d.pdiag[i]);
    }
    solo_sum<3>(v, sh);
    if (threadIdx.x == 0) {
        s.xbar = xbar;
        s.nf = v[0] + 1e-20;
        s.nres0 = v[1] / s.nf;
        s.nres = s.nres0;
        s.tol_eff = fmax(s.tol, s.rel_tol * s.nres0);
        s.iters = 0;
        s.done = 0;
        s.status = FVM_OK;
        s.first = 1;
        s.beta = 0.0;
        if (!isfinite(s.nres0)) set_done(s, FVM_ENUMERIC);
        else if (s.nres0 <= s.tol_eff) set_done(s, FVM_OK);
        else if (!(v[2] > 0.0) || !isfinite(v[2])) { set_done(s, FVM_ENUMERIC); s.iters = 1; }
        else s.rho = v[2];
    }
    __syncthreads();
    if (!mixed) {
        const CGArr<double> a = cg_arrays<double>(d, 0);
        for (long it = 0; it <= (long)d.p_max_iter && !s.done; ++it) solo_cg_iteration<double>(d, sh, a, s);
    } else {
        // k_rr_start: r32 = r64, rho = r32.(r32/diag32)
        if (!s.done) {
            double rho[1] = {0.0};
            SOLO_FOR(i, d.N) {
                const float r = (float)d.r[i];
                d.f_r[i] = r;
                rho[0] += (double)r * (double)(r / d.f_pdiag[i]);
            }
            solo_sum<1>(rho, sh);
            if (threadIdx.x == 0) {
                s.scale = s.nres;
                if (!(rho[0] > 0.0) || !isfinite(rho[0])) { set_done(s, FVM_ENUMERIC); s.iters = 1; }
                else s.rho = rho[0];
            }
            __syncthreads();
        }
        // iterations with a replacement check after every fourth, as the
        // launched driver enqueues them (a paused recurrence waits for it)
        constexpr int kReplaceEvery = 4;
        const CGArr<float> a = cg_arrays<float>(d, 0);
        const long limit = ((long)d.p_max_iter + 2) * kReplaceEvery;
        for (long k = 0; k < limit && s.done != 1; ++k) {
            if (!s.done) solo_cg_iteration<float>(d, sh, a, s);
            if ((k + 1) % kReplaceEvery == 0) solo_rr_replace(d, sh, s);
        }
    }
    if (threadIdx.x == 0 && s.done != 1) set_done(s, FVM_ENUMERIC);
    __syncthreads();
}

__device__ __forceinline__ void worst_status(int32_t &acc, int32_t s)
{
    if (s < 0) { if (acc >= 0 || s < acc) acc = s; }
    else if (acc >= 0 && s > acc) acc = s;
}

// n_steps PISO steps of case blockIdx.x of the batch (orthogonal mesh)
__global__ void __launch_bounds__(kSolo) k_solo_piso(Batch bt, int n_steps, int n_corr)
{
    __shared__ SoloShared sh;
    __shared__ DevCase sdc;
    if ((int)blockIdx.x >= bt.n) return;
    // the case descriptor in LDS: the step reads its fields after its own
    // stores throughout (the descriptor's memory could alias them), and from
    // LDS such a re-read is an LDS access instead of a memory round trip
    {
        static_assert(sizeof(DevCase) % 4 == 0, "the descriptor is copied in words");
        const unsigned int *src = reinterpret_cast<const unsigned int *>(bt.dc[blockIdx.x]);
        unsigned int *dst = reinterpret_cast<unsigned int *>(&sdc);
        for (int t = (int)threadIdx.x; t < (int)(sizeof(DevCase) / 4); t += kSolo) dst[t] = src[t];
        __syncthreads();
    }
    const DevCase &d = sdc;
    const bool mixed = d.f_x != nullptr;
    const long N = d.N, F = d.F;
    int32_t worst = FVM_OK;
    int steps_done = 0, failed = 0, np = 0;
    for (int step = 0; step < n_steps; ++step) {
        // start-of-step copies for a rollback (k_save)
        SOLO_FOR(t, (int)(4 * N + F)) {
            if (t < 3 * N) d.U_save[t] = d.U[t];
            else if (t < 4 * N) d.p_save[t - 3 * N] = d.p[t - 3 * N];
            else d.phi_save[t - 4 * N] = d.phi[t - 4 * N];
        }
        __syncthreads();
        // momentum predictor
        SOLO_FOR(f, d.Fi) el_mom_face(d, f);
        __syncthreads();
        SOLO_FOR(i, d.N) el_mom_cell(d, i, 0);
        __syncthreads();
        solo_momentum(d, sh, mixed);
        int32_t st = FVM_OK;
        for (int c = 0; c < 3; ++c) worst_status(st, sh.ks[c].status);
        if (threadIdx.x == 0)
            for (int c = 0; c < 3; ++c) sh.rec[c] = sh.ks[c];
        np = 0;
        if (st >= 0)
            for (int corr = 0; corr < n_corr; ++corr) {
                SOLO_FOR(i, d.N) el_hbya(d, i, 0);
                __syncthreads();
                SOLO_FOR(f, d.F) el_p_face(d, f);
                __syncthreads();
                SOLO_FOR(i, d.N) el_p_cell(d, i, 1);
                __syncthreads();
                solo_pressure(d, sh, mixed);
                if (threadIdx.x == 0) sh.rec[3 + np] = sh.ks[3];
                ++np;
                worst_status(st, sh.ks[3].status);
                if (st < 0) break;
                SOLO_FOR(f, d.F) el_flux_corr(d, f);
                __syncthreads();
                SOLO_FOR(i, d.N) el_U_corr(d, i);
                __syncthreads();
            }
        worst_status(worst, st);
        if (st < 0) {
            // roll the case back to the start of the failing step
            __syncthreads();
            SOLO_FOR(t, (int)(4 * N + F)) {
                if (t < 3 * N) d.U[t] = d.U_save[t];
                else if (t < 4 * N) d.p[t - 3 * N] = d.p_save[t - 3 * N];
                else d.phi[t - 4 * N] = d.phi_save[t - 4 * N];
            }
            failed = 1;
            break;
        }
        ++steps_done;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int k = 0; k < 3 + np && k < kNumKs - 1; ++k) d.ks[k] = sh.rec[k];
        KState m{};
        m.iters = np;
        m.status = worst;
        m.done = steps_done;
        m.first = failed;
        d.ks[kNumKs - 1] = m;
    }
}

// ---------------------------------------------------------------------------
// Operators one at a time (the assembly set of the paper's Table 3 plus the
// matrix products), in the solver's face-major layout and in the paper's
// hybrid layout (Section 3.1), for comparing the two
// ---------------------------------------------------------------------------

// caller face order -> canonical order; oriented values change sign where
// the caller's orientation is reversed
__global__ void k_faces_in(Batch bt, const double *__restrict__ uv, double *__restrict__ out, int oriented)
{
    CASE_OF(bt);
    const int f = K.raw * kBlock + threadIdx.x;
    if (f >= d.F) return;
    out[f] = f < d.Fi ? (oriented ? (double)d.face_sign[f] : 1.0) * uv[d.face_user[f]] : uv[f];
}

// face-major Gauss gradient: the solver's gather
__global__ void k_op_grad(Batch bt, const double *__restrict__ x, double *__restrict__ g)
{
    CASE_OF(bt);
    const int i = K.raw * kBlock + threadIdx.x;
    if (i >= d.N) return;
    double g0, g1, g2;
    gauss_sum(d, i, x, d.patch_pk, d.patch_pv, 1, g0, g1, g2);
    const double V = d.V[i];
    const long N = d.N;
    g[i] = g0 / V; g[N + i] = g1 / V; g[2 * N + i] = g2 / V;
}

// face-major divergence of a canonical face flux (phiH): owned faces out,
// neighbour-side faces in, non-EMPTY boundary faces out
__global__ void k_op_div(Batch bt, double *__restrict__ out)
{
    CASE_OF(bt);
    const int i = K.raw * kBlock + threadIdx.x;
    if (i >= d.N) return;
    const double *__restrict__ ph = d.phiH;
    double sum = 0.0;
    for (int f = d.own_start[i]; f < d.own_start[i + 1]; ++f) sum += ph[f];
    for (int k = d.nbr_start[i]; k < d.nbr_start[i + 1]; ++k) sum -= ph[d.losort[k]];
    for (int k = d.bnd_start[i]; k < d.bnd_start[i + 1]; ++k) {
        const int b = d.bnd_list[k];
        if (d.patch_pk[d.bpatch[b]] != FVM_BC_EMPTY) sum += ph[d.Fi + b];
    }
    out[i] = sum;
}

// face-major A x on the sliced-ELL copy (one block per slice), no dot
__global__ void __launch_bounds__(kBlock) k_op_spmv(Batch bt, const double *__restrict__ x, double *__restrict__ y)
{
    CASE_OF(bt);
    const int i = K.raw * kBlock + threadIdx.x;
    if (K.raw * kBlock >= d.N) return;
    const CGArr<double> v{d.pdiag, d.poff, nullptr, d.sell_val, nullptr, nullptr, const_cast<double *>(x), y, nullptr,
                          nullptr};
    if (i < d.N) (void)spmv_cell<double, 0>(d, v, K.raw, i);
}

// hybrid layout: device position of the entry whose transpose code is Jc in
// row j's slot (a slot of B, or -1 - c for position c of C)
__device__ __forceinline__ long hy_tpos(const DevCase &d, int j, int Jc)
{
    return Jc >= 0 ? (long)Jc * d.N + j : (long)d.hy_K * d.N + (-1 - Jc);
}

// face data of canonical internal faces into their owner-side entries
__global__ void k_hy_geom(Batch bt)
{
    CASE_OF(bt);
    const int f = K.raw * kBlock + threadIdx.x;
    if (f >= d.Fi) return;
    const long p = d.hy_locO[f];
    d.hy_Sx[p] = d.Sx[f]; d.hy_Sy[p] = d.Sy[f]; d.hy_Sz[p] = d.Sz[f];
    d.hy_w[p] = d.w[f]; d.hy_dl[p] = d.dl[f];
}

// caller face values -> owner-side entries of the layout
__global__ void k_hy_faces_in(Batch bt, const double *__restrict__ uv, double *__restrict__ dst, int oriented)
{
    CASE_OF(bt);
    const int f = K.raw * kBlock + threadIdx.x;
    if (f >= d.Fi) return;
    dst[d.hy_locO[f]] = (oriented ? (double)d.face_sign[f] : 1.0) * uv[d.face_user[f]];
}

// matrix values from [diag N | upper Fi | lower Fi] in caller order
__global__ void k_hy_setmat(Batch bt, const double *__restrict__ in)
{
    CASE_OF(bt);
    const int t = K.raw * kBlock + threadIdx.x;
    if (t < d.N) d.hy_V[d.hy_dpos[t]] = in[t];
    if (t < d.Fi) {
        const int u = d.face_user[t];
        const double up = in[d.N + u], lo = in[(long)d.N + d.Fi + u];
        const bool same = d.face_sign[t] > 0;
        d.hy_V[d.hy_locO[t]] = same ? up : lo;
        d.hy_V[d.hy_locN[t]] = same ? lo : up;
    }
}

// Row i of the hybrid layout, entries in ascending column order (B, then
// C); for each off-diagonal entry the face data sits at the entry itself
// when i owns the face (j > i) and at the transposed entry otherwise.
// Gauss gradient of x
__global__ void k_hy_grad(Batch bt, const double *__restrict__ x, double *__restrict__ g)
{
    CASE_OF(bt);
    const int i = K.raw * kBlock + threadIdx.x;
    if (i >= d.N) return;
    const long N = d.N, KN = (long)d.hy_K * N;
    const double xi = x[i];
    double g0 = 0.0, g1 = 0.0, g2 = 0.0;
    auto face = [&](long own_pos, long tr_pos, int j) {
        const bool owner = j > i;
        const long p = owner ? own_pos : tr_pos;
        const double w = d.hy_w[p];
        const double pf = owner ? w * xi + (1.0 - w) * x[j] : w * x[j] + (1.0 - w) * xi;
        const double sg = owner ? 1.0 : -1.0;
        g0 += sg * d.hy_Sx[p] * pf; g1 += sg * d.hy_Sy[p] * pf; g2 += sg * d.hy_Sz[p] * pf;
    };
    for (int k = 0; k < d.hy_K; ++k) {
        const long e = (long)k * N + i;
        const int j = d.hy_I[e];
        if (j != i) face(e, j > i ? e : hy_tpos(d, j, d.hy_J[e]), j);
    }
    for (int c = d.hy_cstart[i]; c < d.hy_cstart[i + 1]; ++c) {
        const int j = d.hy_ccol[c];
        if (j != i) face(KN + c, d.hy_ctrpos[c], j);
    }
    for (int k = d.bnd_start[i]; k < d.bnd_start[i + 1]; ++k) {
        const int b = d.bnd_list[k], f = d.Fi + b, pt = d.bpatch[b], kind = d.patch_pk[pt];
        if (kind == FVM_BC_EMPTY) continue;
        const double pf = kind == FVM_BC_FIXED ? d.patch_pv[pt] : xi;
        g0 += d.Sx[f] * pf; g1 += d.Sy[f] * pf; g2 += d.Sz[f] * pf;
    }
    const double V = d.V[i];
    g[i] = g0 / V; g[N + i] = g1 / V; g[2 * N + i] = g2 / V;
}

// divergence of the flux held in the layout (hy_phi) plus the canonical
// boundary fluxes (phiH)
__global__ void k_hy_div(Batch bt, double *__restrict__ out)
{
    CASE_OF(bt);
    const int i = K.raw * kBlock + threadIdx.x;
    if (i >= d.N) return;
    const long N = d.N, KN = (long)d.hy_K * N;
    double sum = 0.0;
    for (int k = 0; k < d.hy_K; ++k) {
        const long e = (long)k * N + i;
        const int j = d.hy_I[e];
        if (j > i) sum += d.hy_phi[e];
        else if (j < i) sum -= d.hy_phi[hy_tpos(d, j, d.hy_J[e])];
    }
    for (int c = d.hy_cstart[i]; c < d.hy_cstart[i + 1]; ++c) {
        const int j = d.hy_ccol[c];
        if (j > i) sum += d.hy_phi[KN + c];
        else if (j < i) sum -= d.hy_phi[d.hy_ctrpos[c]];
    }
    for (int k = d.bnd_start[i]; k < d.bnd_start[i + 1]; ++k) {
        const int b = d.bnd_list[k];
        if (d.patch_pk[d.bpatch[b]] != FVM_BC_EMPTY) sum += d.phiH[d.Fi + b];
    }
    out[i] = sum;
}

// pressure Laplacian into the layout's values: off-diagonal -gamma dl, the
// diagonal their negated sum plus the FIXED-p boundary terms and the pin
__global__ void k_hy_lap(Batch bt)
{
    CASE_OF(bt);
    const int i = K.raw * kBlock + threadIdx.x;
    if (i >= d.N) return;
    const long N = d.N, KN = (long)d.hy_K * N, dp = d.hy_dpos[i];
    double dg = 0.0;
    for (int k = 0; k < d.hy_K; ++k) {
        const long e = (long)k * N + i;
        const int j = d.hy_I[e];
        if (j == i) {
            if (e != dp) d.hy_V[e] = 0.0;   // unused slot
            continue;
        }
        const long p = j > i ? e : hy_tpos(d, j, d.hy_J[e]);
        const double a = d.hy_g[p] * d.hy_dl[p];
        d.hy_V[e] = -a;
        dg += a;
    }
    for (int c = d.hy_cstart[i]; c < d.hy_cstart[i + 1]; ++c) {
        const int j = d.hy_ccol[c];
        if (j == i) continue;
        const long p = j > i ? KN + c : d.hy_ctrpos[c];
        const double a = d.hy_g[p] * d.hy_dl[p];
        d.hy_V[KN + c] = -a;
        dg += a;
    }
    for (int k = d.bnd_start[i]; k < d.bnd_start[i + 1]; ++k) {
        const int b = d.bnd_list[k], f = d.Fi + b;
        if (d.patch_pk[d.bpatch[b]] == FVM_BC_FIXED) dg += d.gam[f] * d.dl[f];
    }
    if (i == d.pin_cell && !d.has_fixed_p) dg = 2.0 * dg;
    d.hy_V[dp] = dg;
}

// y = A x (row access: V, I) or A^T x (column access: the value of the
// transposed entry, found through J)
__global__ void k_hy_spmv(Batch bt, const double *__restrict__ x, double *__restrict__ y, int transpose)
{
    CASE_OF(bt);
    const int i = K.raw * kBlock + threadIdx.x;
    if (i >= d.N) return;
    const long N = d.N, KN = (long)d.hy_K * N;
    double acc = 0.0;
    if (!transpose) {
        for (int k = 0; k < d.hy_K; ++k) {
            const long e = (long)k * N + i;
            acc += d.hy_V[e] * x[d.hy_I[e]];
        }
        for (int c = d.hy_cstart[i]; c < d.hy_cstart[i + 1]; ++c) acc += d.hy_V[KN + c] * x[d.hy_ccol[c]];
    } else {
        for (int k = 0; k < d.hy_K; ++k) {
            const long e = (long)k * N + i;
            const int j = d.hy_I[e];
            acc += d.hy_V[hy_tpos(d, j, d.hy_J[e])] * x[j];
        }
        for (int c = d.hy_cstart[i]; c < d.hy_cstart[i + 1]; ++c) acc += d.hy_V[d.hy_ctrpos[c]] * x[d.hy_ccol[c]];
    }
    y[i] = acc;
}

// ---------------------------------------------------------------------------
// Aggregation AMG preconditioner (pressure CG): one V-cycle per application.
// Level l restricts to level l + 1 by summing over each aggregate, and
// prolongs by copying an aggregate's value to its cells.  On the way down a
// level smooths once from zero (x = w D^-1 b) and forms its residual; on the
// way up it adds the coarse correction and smooths once more.  On the
// coarse levels both steps are single fused kernels that evaluate the
// neighbours' x on the fly from the same expression that stores it; the
// finest level writes x first and then runs the solver's sliced-ELL SpMV
// row code (coalesced, mirrored lower slots).  The coarsest level applies a
// dense inverse built at the start of each solve.
// These kernels run on single-case groups, with explicit grids.
// ---------------------------------------------------------------------------
constexpr double kAmgOmega = 2.0 / 3.0;

__global__ void __launch_bounds__(kBlock) k_amg_galerkin(const DevCase *dc, int l)
{
    const DevCase &d = *dc;
    if (d.ks[3].done) return;
    const AmgLevel &C = d.amg[l], &F = d.amg[l - 1];
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t < C.n) {
        double a = 0.0;
        for (int k = C.mstart[t]; k < C.mstart[t + 1]; ++k) a += F.diag[C.members[k]];
        for (int k = C.istart[t]; k < C.istart[t + 1]; ++k) a += 2.0 * F.offd[C.inner[k]];
        C.diag[t] = a;
    }
    if (t < C.nf) {
        double a = 0.0;
        for (int k = C.cstart[t]; k < C.cstart[t + 1]; ++k) a += F.offd[C.cfaces[k]];
        C.offd[t] = a;
    }
}

// inverse of the coarsest matrix by Gauss-Jordan elimination in place (the
// matrix is symmetric positive definite: no pivoting), one block
__global__ void __launch_bounds__(kBlock) k_amg_cinv(const DevCase *dc)
{
    const DevCase &d = *dc;
    if (d.ks[3].done) return;
    const AmgLevel &C = d.amg[d.amg_nl - 1];
    const int n = C.n, t = threadIdx.x;
    double *A = d.amg_cinv;
    __shared__ double fcol[kAmgDenseMax];
    for (long e = t; e < (long)n * n; e += kBlock) A[e] = 0.0;
    __syncthreads();
    for (int i = t; i < n; i += kBlock) A[(long)i * n + i] = C.diag[i];
    for (int f = t; f < C.nf; f += kBlock) {
        A[(long)C.own[f] * n + C.nei[f]] = C.offd[f];
        A[(long)C.nei[f] * n + C.own[f]] = C.offd[f];
    }
    __syncthreads();
    for (int k = 0; k < n; ++k) {
        const double piv = A[(long)k * n + k];
        __syncthreads();
        for (int j = t; j < n; j += kBlock) A[(long)k * n + j] = j == k ? 1.0 / piv : A[(long)k * n + j] / piv;
        for (int i = t; i < n; i += kBlock) fcol[i] = i == k ? 0.0 : A[(long)i * n + k];
        __syncthreads();
        for (long e = t; e < (long)n * n; e += kBlock) {
            const int i = (int)(e / n), j = (int)(e % n);
            if (i == k) continue;
            A[e] = j == k ? -fcol[i] * A[(long)k * n + k] : A[e] - fcol[i] * A[(long)k * n + j];
        }
        __syncthreads();
    }
}

// x = w b / diag and r = b - A x (neighbours' x from their b and diag)
__global__ void __launch_bounds__(kBlock) k_amg_down(const DevCase *dc, int l)
{
    const DevCase &d = *dc;
    if (d.ks[3].done) return;
    const AmgLevel &L = d.amg[l];
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= L.n) return;
    const double bi = L.b[i], xi = kAmgOmega * bi / L.diag[i];
    L.x[i] = xi;
    double ax = L.diag[i] * xi;
    for (int f = L.own_start[i]; f < L.own_start[i + 1]; ++f) {
        const int j = L.nei[f];
        ax += L.offd[f] * (kAmgOmega * L.b[j] / L.diag[j]);
    }
    for (int k = L.nbr_start[i]; k < L.nbr_start[i + 1]; ++k) {
        const int f = L.losort[k], j = L.own[f];
        ax += L.offd[f] * (kAmgOmega * L.b[j] / L.diag[j]);
    }
    L.r[i] = bi - ax;
}

// coarse right-hand side: sum of the fine residuals over each aggregate
__global__ void __launch_bounds__(kBlock) k_amg_restrict(const DevCase *dc, int l)
{
    const DevCase &d = *dc;
    if (d.ks[3].done) return;
    const AmgLevel &C = d.amg[l], &F = d.amg[l - 1];
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= C.n) return;
    double a = 0.0;
    for (int k = C.mstart[t]; k < C.mstart[t + 1]; ++k) a += F.r[C.members[k]];
    C.b[t] = a;
}

// coarsest level: out = A^-1 b
__global__ void __launch_bounds__(kBlock) k_amg_coarse(const DevCase *dc)
{
    const DevCase &d = *dc;
    if (d.ks[3].done) return;
    const AmgLevel &C = d.amg[d.amg_nl - 1];
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= C.n) return;
    const double *row = d.amg_cinv + (long)i * C.n;
    double a = 0.0;
    for (int j = 0; j < C.n; ++j) a += row[j] * C.b[j];
    C.out[i] = a;
}

// x' = x + P xc, out = x' + w (b - A x') / diag (neighbours' x' on the fly)
__global__ void __launch_bounds__(kBlock) k_amg_up(const DevCase *dc, int l)
{
    const DevCase &d = *dc;
    if (d.ks[3].done) return;
    const AmgLevel &L = d.amg[l];
    const double *__restrict__ xc = d.amg[l + 1].out;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= L.n) return;
    const double xi = L.x[i] + xc[L.agg[i]];
    double ax = L.diag[i] * xi;
    for (int f = L.own_start[i]; f < L.own_start[i + 1]; ++f) {
        const int j = L.nei[f];
        ax += L.offd[f] * (L.x[j] + xc[L.agg[j]]);
    }
    for (int k = L.nbr_start[i]; k < L.nbr_start[i + 1]; ++k) {
        const int f = L.losort[k], j = L.own[f];
        ax += L.offd[f] * (L.x[j] + xc[L.agg[j]]);
    }
    L.out[i] = xi + kAmgOmega * (L.b[i] - ax) / L.diag[i];
}

// Small coarse levels: a thread per row would walk its faces one dependent
// load after another with few waves to hide the latency.  There a wave
// takes a row, its lanes split the row's faces (or the aggregate's members)
// and a fixed shuffle tree sums them.  Larger levels keep a thread per row
// (a wave per row would leave most lanes idle).
constexpr int kAmgWaveRows = 32768;   // levels with at most this many rows
constexpr int kRowsPerBlock = kBlock / 64;

__device__ __forceinline__ double wave_sum64(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__global__ void __launch_bounds__(kBlock) k_amg_down_w(const DevCase *dc, int l)
{
    const DevCase &d = *dc;
    if (d.ks[3].done) return;
    const AmgLevel &L = d.amg[l];
    const int i = blockIdx.x * kRowsPerBlock + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (i >= L.n) return;   // the whole wave
    const int o0 = L.own_start[i], no = L.own_start[i + 1] - o0;
    const int n0 = L.nbr_start[i], nn = L.nbr_start[i + 1] - n0;
    double acc = 0.0;
    for (int t = lane; t < no + nn; t += 64) {
        const int f = t < no ? o0 + t : L.losort[n0 + t - no];
        const int j = t < no ? L.nei[f] : L.own[f];
        acc += L.offd[f] * (kAmgOmega * L.b[j] / L.diag[j]);
    }
    acc = wave_sum64(acc);
    if (lane == 0) {
        const double bi = L.b[i], xi = kAmgOmega * bi / L.diag[i];
        L.x[i] = xi;
        L.r[i] = bi - (L.diag[i] * xi + acc);
    }
}

__global__ void __launch_bounds__(kBlock) k_amg_restrict_w(const DevCase *dc, int l)
{
    const DevCase &d = *dc;
    if (d.ks[3].done) return;
    const AmgLevel &C = d.amg[l], &F = d.amg[l - 1];
    const int t = blockIdx.x * kRowsPerBlock + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (t >= C.n) return;
    double a = 0.0;
    for (int k = C.mstart[t] + lane; k < C.mstart[t + 1]; k += 64) a += F.r[C.members[k]];
    a = wave_sum64(a);
    if (lane == 0) C.b[t] = a;
}

__global__ void __launch_bounds__(kBlock) k_amg_up_w(const DevCase *dc, int l)
{
    const DevCase &d = *dc;
    if (d.ks[3].done) return;
    const AmgLevel &L = d.amg[l];
    const double *__restrict__ xc = d.amg[l + 1].out;
    const int i = blockIdx.x * kRowsPerBlock + (threadIdx.x >> 6), lane = threadIdx.x & 63;
    if (i >= L.n) return;
    const int o0 = L.own_start[i], no = L.own_start[i + 1] - o0;
    const int n0 = L.nbr_start[i], nn = L.nbr_start[i + 1] - n0;
    double acc = 0.0;
    for (int t = lane; t < no + nn; t += 64) {
        const int f = t < no ? o0 + t : L.losort[n0 + t - no];
        const int j = t < no ? L.nei[f] : L.own[f];
        acc += L.offd[f] * (L.x[j] + xc[L.agg[j]]);
    }
    acc = wave_sum64(acc);
    if (lane == 0) {
        const double xi = L.x[i] + xc[L.agg[i]];
        L.out[i] = xi + kAmgOmega * (L.b[i] - (L.diag[i] * xi + acc)) / L.diag[i];
    }
}

// The smallest levels and the coarse solve in one launch.  Below a few
// hundred rows each of the kernels above costs a launch and a couple of
// dependent global-memory round trips whatever its size, so the levels
// l0 .. nl - 1 whose structure fits in LDS run in one block.  Once per
// solve (after the Galerkin products) k_amg_tail_pack writes their
// structure and matrix values into an HBM image laid out exactly as the
// LDS; each cycle then stages that image and level l0's right-hand side
// with one round of independent 16-byte loads, smooths, restricts, solves
// and prolongs in LDS, and writes only the corrected x of level l0.  The
// arithmetic is that of k_amg_down, k_amg_restrict, k_amg_coarse and
// k_amg_up (the coarse product split over a wave's lanes).
constexpr int kAmgTailThreads = 1024;
constexpr int kAmgTailWords = kAmgTailLds / 16 / kAmgTailThreads;   // 16-byte loads per thread

// LDS carving: consecutive arrays, each rounded up to 16 bytes.  The host
// walks the same sequence with a null base to size the launch.
struct LdsBump {
    char *base;   // null when only sizing
    long off;
    template <class T> __host__ __device__ T *take(long n)
    {
        T *r = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += (n * (long)sizeof(T) + 15) / 16 * 16;
        return r;
    }
};

struct AmgTailLevel {
    double *diag, *offd, *b, *x, *r;   // r holds out on the way up
    int32_t *os, *ns, *nei, *own, *losort, *agg, *cmstart, *cmembers;
};

// level l of the tail (l < nl - 1 has the full structure; the coarsest level
// only b and out)
__host__ __device__ inline AmgTailLevel amg_tail_carve(LdsBump &bp, const int32_t *n, const int32_t *nf, int l, int nl)
{
    AmgTailLevel t{};
    const long m = n[l];
    t.b = bp.take<double>(m);
    t.r = bp.take<double>(m);
    if (l < nl - 1) {
        const long f = nf[l];
        t.diag = bp.take<double>(m);
        t.x = bp.take<double>(m);
        t.offd = bp.take<double>(f);
        t.os = bp.take<int32_t>(m + 1);
        t.ns = bp.take<int32_t>(m + 1);
        t.nei = bp.take<int32_t>(f);
        t.own = bp.take<int32_t>(f);
        t.losort = bp.take<int32_t>(f);
        t.agg = bp.take<int32_t>(m);
        t.cmstart = bp.take<int32_t>(n[l + 1] + 1);
        t.cmembers = bp.take<int32_t>(m);
    }
    return t;
}

// LDS bytes of the tail from level l0, or -1 when it does not fit
__host__ inline long amg_tail_bytes(const int32_t *n, const int32_t *nf, int l0, int nl)
{
    LdsBump bp{nullptr, 0};
    for (int l = l0; l < nl; ++l) amg_tail_carve(bp, n, nf, l, nl);
    return bp.off <= kAmgTailLds ? bp.off : -1;
}

// the LDS arrays of tail level l for an image at base (carved again where
// needed: a handful of scalar operations, and no per-lane pointer table)
__device__ inline AmgTailLevel amg_tail_level(const DevCase &d, char *base, int l0, int l)
{
    LdsBump bp{base, 0};
    for (int k = l0; k < l; ++k) amg_tail_carve(bp, d.amg_n, d.amg_nf, k, d.amg_nl);
    return amg_tail_carve(bp, d.amg_n, d.amg_nf, l, d.amg_nl);
}

template <class T>
__device__ __forceinline__ void tail_copy(T *dst, const T *__restrict__ src, long n)
{
    for (long k = threadIdx.x; k < n; k += kAmgTailThreads) dst[k] = src[k];
}

// once per solve: the HBM image of the tail levels (b and r stay unset)
__global__ void __launch_bounds__(kAmgTailThreads) k_amg_tail_pack(const DevCase *dc, int l0)
{
    const DevCase &d = *dc;
    if (d.ks[3].done) return;
    char *img = reinterpret_cast<char *>(d.amg_img);
    for (int l = l0; l < d.amg_nl - 1; ++l) {
        const AmgTailLevel t = amg_tail_level(d, img, l0, l);
        const AmgLevel &L = d.amg[l], &C = d.amg[l + 1];
        const int m = L.n, f = L.nf;
        tail_copy(t.diag, L.diag, m);
        tail_copy(t.offd, L.offd, f);
        tail_copy(t.os, L.own_start, m + 1);
        tail_copy(t.ns, L.nbr_start, m + 1);
        tail_copy(t.nei, L.nei, f);
        tail_copy(t.own, L.own, f);
        tail_copy(t.losort, L.losort, f);
        tail_copy(t.agg, L.agg, m);
        tail_copy(t.cmstart, C.mstart, C.n + 1);
        tail_copy(t.cmembers, C.members, m);
    }
}

// bytes: the image size (amg_tail_bytes), at most kAmgTailLds; src: the
// image; gb, gout: level l0's b and out; cinv: the coarse inverse; n0, mc:
// the sizes of level l0 and of the coarsest level.  The buffers come as
// arguments so that their loads leave before the stop flag is read.
__global__ void __launch_bounds__(kAmgTailThreads)
k_amg_tail(const DevCase *dc, int l0, int bytes, const int4 *__restrict__ src, const double *__restrict__ gb,
           double *__restrict__ gout, const double *__restrict__ cinv, int n0, int mc)
{
    const DevCase &d = *dc;
    extern __shared__ __align__(16) char amg_lds[];
    const int tid = threadIdx.x;
    const bool stop = d.ks[3].done;
    const bool cpre = mc <= 2 * (kAmgTailThreads / 64);
    double cv0 = 0.0, cv1 = 0.0;
    {
        // level l0's b opens the image; the rest comes from the packed copy.
        // Every load is issued before the first LDS store.
        const int w0 = (n0 * 8 + 15) / 16, w1 = bytes / 16;
        int4 v[kAmgTailWords];
        double bv[2];
        if (cpre) {
            // the coarse inverse's entries this lane multiplies (rows tid / 64
            // and tid / 64 + 16 of at most 32, one column each)
            const int i0 = tid >> 6, j = tid & 63;
            if (j < mc && i0 < mc) cv0 = cinv[(long)i0 * mc + j];
            if (j < mc && i0 + kAmgTailThreads / 64 < mc) cv1 = cinv[(long)(i0 + kAmgTailThreads / 64) * mc + j];
        }
#pragma unroll
        for (int k = 0; k < kAmgTailWords; ++k) {
            const int w = w0 + tid + k * kAmgTailThreads;
            if (w < w1) v[k] = src[w];
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int i = tid + k * kAmgTailThreads;
            if (i < n0) bv[k] = gb[i];
        }
        int4 *dst = reinterpret_cast<int4 *>(amg_lds);
        double *lb = reinterpret_cast<double *>(amg_lds);
#pragma unroll
        for (int k = 0; k < kAmgTailWords; ++k) {
            const int w = w0 + tid + k * kAmgTailThreads;
            if (w < w1) dst[w] = v[k];
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int i = tid + k * kAmgTailThreads;
            if (i < n0) lb[i] = bv[k];
        }
        for (int i = tid + 2 * kAmgTailThreads; i < n0; i += kAmgTailThreads) lb[i] = gb[i];
    }
    if (stop) return;   // the whole block
    const int nl = d.amg_nl;
    auto level = [&](int l) { return amg_tail_level(d, amg_lds, l0, l); };
    __syncthreads();

    // Rows of a level go to groups of G lanes (G a power of two, the largest
    // with G * rows <= the block, at most 64); a group's lanes split the
    // row's faces and a shuffle tree sums them.  x is stored in a pass of
    // its own so the face loops read it instead of recomputing it.
    auto group = [](int m) {
        int g = 1;
        while (g < 64 && 2 * g * m <= kAmgTailThreads) g *= 2;
        return g;
    };
    auto gsum = [](double v, int g) {
        for (int o = g >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        return v;
    };
    // A x without the diagonal: faces of row i, split over the group
    auto offdiag = [](const AmgTailLevel &t, const double *x, int i, int sub, int g) {
        const int o0 = t.os[i], no = t.os[i + 1] - o0;
        const int n0 = t.ns[i], nn = t.ns[i + 1] - n0;
        double a = 0.0;
        for (int k = sub; k < no + nn; k += g) {
            const int f = k < no ? o0 + k : t.losort[n0 + k - no];
            const int j = k < no ? t.nei[f] : t.own[f];
            a += t.offd[f] * x[j];
        }
        return a;
    };

    // down: x = w b / diag, r = b - A x, restrict
    for (int l = l0; l < nl - 1; ++l) {
        const AmgTailLevel t = level(l);
        const int m = d.amg_n[l], g = group(m), sub = tid & (g - 1);
        for (int i = tid; i < m; i += kAmgTailThreads) t.x[i] = kAmgOmega * t.b[i] / t.diag[i];
        __syncthreads();
        for (int base = 0; base < m; base += kAmgTailThreads / g) {
            const int i = base + tid / g;
            const double a = gsum(i < m ? offdiag(t, t.x, i, sub, g) : 0.0, g);
            if (i < m && sub == 0) t.r[i] = t.b[i] - (t.diag[i] * t.x[i] + a);
        }
        __syncthreads();
        const int mn = d.amg_n[l + 1], gc = group(mn), subc = tid & (gc - 1);
        double *cb = level(l + 1).b;
        for (int base = 0; base < mn; base += kAmgTailThreads / gc) {
            const int c = base + tid / gc;
            double a = 0.0;
            if (c < mn)
                for (int k = t.cmstart[c] + subc; k < t.cmstart[c + 1]; k += gc) a += t.r[t.cmembers[k]];
            a = gsum(a, gc);
            if (c < mn && subc == 0) cb[c] = a;
        }
        __syncthreads();
    }

    // coarsest: out = A^-1 b, a wave per row, lanes split the row
    {
        const AmgTailLevel t = level(nl - 1);
        const int lane = tid & 63;
        for (int i = tid >> 6, k = 0; i < mc; i += kAmgTailThreads / 64, ++k) {
            double a = 0.0;
            if (cpre) {
                if (lane < mc) a = (k == 0 ? cv0 : cv1) * t.b[lane];
            } else {
                const double *row = d.amg_cinv + (long)i * mc;
                for (int j = lane; j < mc; j += 64) a += row[j] * t.b[j];
            }
            a = wave_sum64(a);
            if (lane == 0) t.r[i] = a;
        }
        __syncthreads();
    }

    // up: x' = x + P xc, out = x' + w (b - A x') / diag; level l0 writes its
    // result to HBM
    for (int l = nl - 2; l >= l0; --l) {
        const AmgTailLevel t = level(l);
        const double *xc = level(l + 1).r;
        const int m = d.amg_n[l], g = group(m), sub = tid & (g - 1);
        for (int i = tid; i < m; i += kAmgTailThreads) t.x[i] += xc[t.agg[i]];
        __syncthreads();
        for (int base = 0; base < m; base += kAmgTailThreads / g) {
            const int i = base + tid / g;
            const double a = gsum(i < m ? offdiag(t, t.x, i, sub, g) : 0.0, g);
            if (i < m && sub == 0) {
                const double xi = t.x[i];
                const double o = xi + kAmgOmega * (t.b[i] - (t.diag[i] * xi + a)) / t.diag[i];
                if (l == l0) gout[i] = o;
                else t.r[i] = o;
            }
        }
        __syncthreads();
    }
}

// rho/beta update from r.z (the value every block has summed)
__device__ __forceinline__ void amg_rho(KState &s, double rz)
{
    if (!(rz > 0.0) || !isfinite(rz)) { set_done(s, FVM_ENUMERIC); s.iters += 1; }
    else if (s.iters == 0) s.rho = rz;
    else {
        s.beta = rz / s.rho;
        s.rho = rz;
    }
}

// The finest level through the sliced-ELL copy of the pressure matrix (the
// solver's SpMV row code: coalesced slot streams, mirrored lower slots):
// the smoothed or corrected x is written out first, then one pass forms
// the residual or the second smoothing step.
__global__ void __launch_bounds__(kBlock) k_amg_x0(Batch bt, int up)
{
    CASE_OF(bt);
    if (d.ks[3].done) return;
    const AmgLevel &L = d.amg[0];
    const double *__restrict__ xc = d.amg[1].out;
    const Range rg = block_range(d.N, K);
    for (int i = rg.beg + threadIdx.x; i < rg.end; i += kBlock)
        L.x[i] = up ? L.x[i] + xc[L.agg[i]] : kAmgOmega * L.b[i] / L.diag[i];
}

// down: r = b - A x; up: z = x + w (b - A x) / diag, with r.z
__global__ void __launch_bounds__(kBlock) k_amg_sell(Batch bt, int up)
{
    CASE_OF(bt);
    if (d.ks[3].done) return;
    const AmgLevel &L = d.amg[0];
    const CGArr<double> v{d.pdiag, d.poff, nullptr, d.sell_val, nullptr, nullptr, L.x, L.r, nullptr, nullptr};
    const Range rg = block_range(d.N, K);
    double acc[1] = {0.0};
    for (int base = rg.beg; base < rg.end; base += kBlock) {
        const int i = base + threadIdx.x;
        if (i >= rg.end) continue;
        (void)spmv_cell<double, 0>(d, v, base / kBlock, i);   // L.r[i] = (A x)_i
        const double bi = L.b[i];
        if (!up) L.r[i] = bi - L.r[i];
        else {
            const double z = L.x[i] + kAmgOmega * (bi - L.r[i]) / L.diag[i];
            L.out[i] = z;
            acc[0] += bi * z;
        }
    }
    if (!up) return;
    __shared__ double tot[1];
    if (reduce_last<1>(acc, d, K, tot) && threadIdx.x == 0) amg_rho(d.ks[3], tot[0]);
}


// rho = r.z after the preconditioner; beta from the previous rho
__global__ void __launch_bounds__(kBlock) k_amg_rz(Batch bt)
{
    CASE_OF(bt);
    if (d.ks[3].done) return;
    const Range rg = block_range(d.N, K);
    double v[1] = {0.0};
    for (int i = rg.beg + threadIdx.x; i < rg.end; i += kBlock) v[0] += d.r[i] * d.z[i];
    __shared__ double tot[1];
    if (reduce_last<1>(v, d, K, tot) && threadIdx.x == 0) amg_rho(d.ks[3], tot[0]);
}

}  // namespace

// ---------------------------------------------------------------------------
// Host side: batch descriptors and launchers
// ---------------------------------------------------------------------------

int blocks_for(int n)
{
    const int g = cdiv(n, kBlock);
    return g < 1 ? 8 : (g + 7) / 8 * 8;
}

int grid_for(int n) { return blocks_for(n); }

void batch_add(BatchSet &bs, const DevCase *dev, const DevCase *host)
{
    const int c = bs.n;
    for (int k = 0; k < SZ_KINDS; ++k) {
        Batch &b = bs.b[k];
        b.dc[c] = dev;
        if (c == 0) b.start[0] = 0;
        int n = host->N > host->Fi ? host->N : host->Fi;
        if (k == SZ_CELL) n = host->N;
        else if (k == SZ_FACE) n = host->F;
        else if (k == SZ_FACEI) n = host->Fi;
        else if (k == SZ_CELL2) n = (host->N + 1) / 2;
        else if (k == SZ_CELL4) n = (host->N + 3) / 4;
        else if (k == SZ_CELL8) n = (host->N + 7) / 8;
        else if (k == SZ_CELL16) n = (host->N + 15) / 16;
        b.start[c + 1] = b.start[c] + blocks_for(n);
        b.n = c + 1;
    }
    bs.host[c] = host;
    bs.n = c + 1;
}

namespace {
template <class... P, class... A>
void run(void (*kern)(Batch, P...), const BatchSet &bs, int kind, hipStream_t s, A... args)
{
    const Batch &b = bs.b[kind];
    hipLaunchKernelGGL(kern, dim3(b.start[b.n]), dim3(kBlock), 0, s, b, static_cast<P>(args)...);
}

struct Prof {
    const char *c;
    hipStream_t s;
    Prof(const char *cls, hipStream_t st) : c(cls), s(st) { prof_begin(c, s); }
    ~Prof() { prof_end(c, s); }
};
}  // namespace

void launch_geometry(const BatchSet &bs, hipStream_t s) { run(k_geometry, bs, SZ_FACE, s); }
void launch_flux_from_U(const BatchSet &bs, hipStream_t s) { run(k_flux_from_U, bs, SZ_FACE, s); }
void launch_U_in(const BatchSet &bs, const double *U, hipStream_t s) { run(k_U_in, bs, SZ_CELL, s, U); }
void launch_U_out(const BatchSet &bs, double *U, hipStream_t s) { run(k_U_out, bs, SZ_CELL, s, U); }
void launch_phi_in(const BatchSet &bs, const double *phi, hipStream_t s) { run(k_phi_in, bs, SZ_FACE, s, phi); }
void launch_phi_out(const BatchSet &bs, double *phi, hipStream_t s) { run(k_phi_out, bs, SZ_FACE, s, phi); }
void launch_gather_faces(const BatchSet &bs, const double *uv, double *out, hipStream_t s)
{
    run(k_gather_faces, bs, SZ_FACE, s, uv, out);
}
void launch_p_system_from_gamma(const BatchSet &bs, const double *gam, const double *rhs, hipStream_t s)
{
    run(k_p_face_gamma, bs, SZ_FACE, s, gam);
    (void)hipMemcpyAsync(bs.host[0]->pb, rhs, sizeof(double) * (size_t)bs.host[0]->N, hipMemcpyDeviceToDevice, s);
    run(k_p_cell, bs, SZ_CELL, s, 0);
}
void launch_init_partials(const BatchSet &bs, hipStream_t s) { run(k_fill_sentinel, bs, SZ_CELL, s); }
void launch_set_patch(const BatchSet &bs, int patch, double u0, double u1, double u2, double pv, hipStream_t s)
{
    run(k_set_patch, bs, SZ_CELL, s, patch, u0, u1, u2, pv);
}

void launch_save(const BatchSet &bs, int restore, hipStream_t s)
{
    // 4N + F words per case: sized by the larger of the two kinds below
    BatchSet t = bs;
    Batch &b = t.b[SZ_CELL];
    b.start[0] = 0;
    for (int c = 0; c < bs.n; ++c) b.start[c + 1] = b.start[c] + blocks_for(4 * bs.host[c]->N + bs.host[c]->F);
    run(k_save, t, SZ_CELL, s, restore);
}

void launch_gradU(const BatchSet &bs, hipStream_t s) { run(k_gradU, bs, SZ_CELL, s); }
void launch_mom_face(const BatchSet &bs, hipStream_t s)
{
    Prof p("mom_face", s);
    run(k_mom_face, bs, SZ_FACEI, s);
}
void launch_mom_cell(const BatchSet &bs, int mode, hipStream_t s)
{
    Prof p("mom_cell", s);
    run(k_mom_cell, bs, SZ_CELL, s, mode);
}
void launch_hbya(const BatchSet &bs, int with_gradp, hipStream_t s)
{
    Prof p("hbya", s);
    run(k_hbya, bs, SZ_CELL, s, with_gradp);
}
void launch_gradp(const BatchSet &bs, hipStream_t s) { run(k_gradp, bs, SZ_CELL, s); }
void launch_p_face(const BatchSet &bs, hipStream_t s)
{
    Prof p("p_face", s);
    run(k_p_face, bs, SZ_FACE, s);
}
void launch_p_cell(const BatchSet &bs, hipStream_t s)
{
    Prof p("p_cell", s);
    run(k_p_cell, bs, SZ_CELL, s, 1);
}
void launch_flux_corr(const BatchSet &bs, hipStream_t s)
{
    Prof p("flux_corr", s);
    run(k_flux_corr, bs, SZ_FACE, s);
}
void launch_p_relax(const BatchSet &bs, hipStream_t s) { run(k_p_relax, bs, SZ_CELL, s); }
void launch_U_corr(const BatchSet &bs, hipStream_t s)
{
    Prof p("U_corr", s);
    run(k_U_corr, bs, SZ_CELL, s);
}

void launch_set_ctl(const BatchSet &bs, int first, int count, int src, double tol, double rel_tol, int max_iter,
                    hipStream_t s)
{
    run(k_set_ctl, bs, SZ_CELL, s, first, count, src, tol, rel_tol, max_iter);
}
void launch_gather_ks(const BatchSet &bs, hipStream_t s) { run(k_gather_ks, bs, SZ_CELL, s); }

void launch_bicg_init(const BatchSet &bs, int stab, hipStream_t s)
{
    run(k_bicg_sumx, bs, SZ_CELL, s);
    run(k_bicg_init, bs, SZ_CELL, s, stab);
}

void launch_bicgstab_iter(const BatchSet &bs, hipStream_t s)
{
    run(k_bs_dir, bs, SZ_CELL, s);
    {
        Prof p("bicgstab_spmv", s);
        run(k_bs_spmv_v, bs, SZ_CELL, s);
    }
    run(k_bs_s, bs, SZ_CELL, s);
    {
        Prof p("bicgstab_spmv", s);
        run(k_bs_spmv_t, bs, SZ_CELL, s);
    }
    run(k_bs_update, bs, SZ_CELL, s);
}

void launch_bicg_iter(const BatchSet &bs, hipStream_t s)
{
    run(k_bicg_dir<double>, bs, SZ_CELL, s);
    {
        Prof p("bicg_spmv", s);
        run(k_bicg_spmv<double>, bs, SZ_CELL, s);
    }
    run(k_bicg_update<double>, bs, SZ_CELL, s);
}

// every case of the batch has 6 slots per sliced-ELL row (hex meshes)
bool sell_w6(const BatchSet &bs)
{
    for (int c = 0; c < bs.n; ++c)
        if (bs.host[c]->sell_W != 6) return false;
    return true;
}

// grid of the CG products: several slices per block
constexpr int kSpmvGrid = SZ_CELL4;
constexpr int kWideDirCells = 4 << 20;   // 2048 blocks of 8 x 256 cells

void launch_pcg_init(const BatchSet &bs, int dic, hipStream_t s)
{
    run(k_sell_fill, bs, SZ_CELL, s);
    run(k_pcg_sumx, bs, SZ_CELL, s);
    run(k_pcg_init, bs, SZ_CELL, s, dic);
}

template <int D>
void dic_sweeps(const BatchSet &bs, int with_setup, hipStream_t s)
{
    if (with_setup) {
        Prof p("dic_setup", s);
        run(k_dic_fill, bs, SZ_CELL, s);
        run(k_dic_sweep<0, D>, bs, SZ_CELL, s);
    }
    {
        Prof p("dic_fwd", s);
        run(k_dic_sweep<1, D>, bs, SZ_CELL, s);
    }
    {
        Prof p("dic_bwd", s);
        run(k_dic_sweep<2, D>, bs, SZ_CELL, s);
    }
}

void launch_dic_precond(const BatchSet &bs, int with_setup, hipStream_t s)
{
    int w = 0;
    for (int c = 0; c < bs.n; ++c) w = std::max(w, std::max(bs.host[c]->dW_lo, bs.host[c]->dW_hi));
    if (w <= 4) dic_sweeps<4>(bs, with_setup, s);
    else dic_sweeps<8>(bs, with_setup, s);
}

void launch_dic_reset(const BatchSet &bs, hipStream_t s) { run(k_dic_reset, bs, SZ_CELL, s); }

void launch_pcg_iter(const BatchSet &bs, int pc, int parity, hipStream_t s)
{
    // Jacobi: the three kernels of an iteration alternate their direction,
    // and iterations alternate which direction comes first, so each kernel
    // walks the cells the other way from its predecessor (DIC and AMG put
    // their own sweeps between the kernels: forward only)
    const int rd = pc == 0 ? parity & 1 : 0, ru = pc == 0 ? 1 - rd : 0;
    {
        Prof p("pcg_dir", s);
        // 8 cells per thread pays once every case has enough blocks to fill
        // the GPU at that width (an element-wise kernel: the result does
        // not depend on the width)
        bool wide = true;
        for (int c = 0; c < bs.n; ++c) wide = wide && bs.host[c]->N >= kWideDirCells;
        if (wide) run(k_cg_dir<double, 8>, bs, SZ_CELL8, s, pc != 0 ? 1 : 0, rd);
        else run(k_cg_dir<double, 4>, bs, SZ_CELL4, s, pc != 0 ? 1 : 0, rd);
    }
    {
        Prof p("pcg_spmv", s);
        if (sell_w6(bs)) run(k_cg_spmv_grp<double, 2>, bs, kSpmvGrid, s, pc != 0 ? 1 : 0, ru);
        else run(k_cg_spmv<double, 0>, bs, kSpmvGrid, s, pc != 0 ? 1 : 0, ru);
    }
    {
        Prof p("pcg_update", s);
        run(k_cg_update<4>, bs, SZ_CELL4, s, pc != 0 ? 1 : 0, rd);
    }
    if (pc == 1) launch_dic_precond(bs, 0, s);
    else if (pc == 2) launch_amg_precond(bs, 0, s);
}

void launch_mx_cvt(const BatchSet &bs, int kind, hipStream_t s) { run(k_mx_cvt, bs, SZ_MAXNF, s, kind); }

void launch_solo_piso(const BatchSet &bs, int n_steps, int n_corr, hipStream_t s)
{
    Prof p("solo_piso", s);
    const Batch &b = bs.b[SZ_CELL];
    hipLaunchKernelGGL(k_solo_piso, dim3((unsigned)b.n), dim3(kSolo), 0, s, b, n_steps, n_corr);
}
void launch_mx_inner_init(const BatchSet &bs, int, hipStream_t s) { run(k_mx_inner_init, bs, SZ_CELL, s); }
void launch_mx_inner_iter(const BatchSet &bs, int, hipStream_t s)
{
    run(k_bicg_dir<float>, bs, SZ_CELL, s);
    {
        Prof p("bicg32_spmv", s);
        run(k_bicg_spmv<float>, bs, SZ_CELL, s);
    }
    run(k_bicg_update<float>, bs, SZ_CELL, s);
}
void launch_bicg_fallback(const BatchSet &bs, hipStream_t s) { run(k_bicg_fallback, bs, SZ_CELL, s); }
void launch_mx_correct_resid(const BatchSet &bs, int, hipStream_t s)
{
    run(k_mx_correct, bs, SZ_CELL, s);
    run(k_mx_resid, bs, SZ_CELL, s);
}

void launch_rr_start(const BatchSet &bs, hipStream_t s)
{
    run(k_mx_cvt, bs, SZ_MAXNF, s, 1);
    run(k_rr_start, bs, SZ_CELL, s);
}

void launch_rr_iter(const BatchSet &bs, int parity, hipStream_t s)
{
    // directions alternate as in launch_pcg_iter
    const int rd = parity & 1, ru = 1 - rd;
    {
        Prof p("pcg32_dir", s);
        run(k_cg_dir<float, 4>, bs, SZ_CELL4, s, 0, rd);
    }
    {
        Prof p("pcg32_spmv", s);
        if (sell_w6(bs)) run(k_cg_spmv<float, 6>, bs, kSpmvGrid, s, 0, ru);
        else run(k_cg_spmv<float, 0>, bs, kSpmvGrid, s, 0, ru);
    }
    {
        Prof p("pcg32_update", s);
        run(k_rr_update<4>, bs, SZ_CELL4, s, rd);
    }
}

void launch_rr_replace(const BatchSet &bs, hipStream_t s)
{
    Prof p("pcg_replace", s);
    run(k_rr_replace, bs, SZ_CELL4, s);
}

// one operator of fvm_case_operator (op validated by the caller); the input
// conversion runs outside the operator's profile class
void launch_operator(const BatchSet &bs, int op, const double *in, double *out, hipStream_t s)
{
    const DevCase &h = *bs.host[0];
    switch (op) {
    case FVM_OP_GRAD: {
        Prof p("op_grad", s);
        run(k_op_grad, bs, SZ_CELL, s, in, out);
        break;
    }
    case FVM_OP_DIV: {
        run(k_faces_in, bs, SZ_FACE, s, in, h.phiH, 1);
        Prof p("op_div", s);
        run(k_op_div, bs, SZ_CELL, s, out);
        break;
    }
    case FVM_OP_LAP: {
        run(k_faces_in, bs, SZ_FACE, s, in, h.gam, 0);
        {
            Prof p("op_lap", s);
            run(k_p_face_gamma, bs, SZ_FACE, s, (const double *)h.gam);
            run(k_p_cell, bs, SZ_CELL, s, 0);
        }
        run(k_sell_fill, bs, SZ_CELL, s);
        (void)hipMemcpyAsync(out, h.pdiag, sizeof(double) * (size_t)h.N, hipMemcpyDeviceToDevice, s);
        break;
    }
    case FVM_OP_SPMV: {
        Prof p("op_spmv", s);
        run(k_op_spmv, bs, SZ_CELL, s, in, out);
        break;
    }
    case FVM_OP_HY_GRAD: {
        Prof p("hy_grad", s);
        run(k_hy_grad, bs, SZ_CELL, s, in, out);
        break;
    }
    case FVM_OP_HY_DIV: {
        run(k_faces_in, bs, SZ_FACE, s, in, h.phiH, 1);
        run(k_hy_faces_in, bs, SZ_FACEI, s, in, h.hy_phi, 1);
        Prof p("hy_div", s);
        run(k_hy_div, bs, SZ_CELL, s, out);
        break;
    }
    case FVM_OP_HY_LAP: {
        run(k_faces_in, bs, SZ_FACE, s, in, h.gam, 0);
        run(k_hy_faces_in, bs, SZ_FACEI, s, in, h.hy_g, 0);
        {
            Prof p("hy_lap", s);
            run(k_hy_lap, bs, SZ_CELL, s);
        }
        (void)hipMemcpyAsync(out, h.hy_V, sizeof(double) * ((size_t)h.hy_K * h.N + h.hy_nC), hipMemcpyDeviceToDevice,
                             s);
        break;
    }
    case FVM_OP_HY_SPMV:
    case FVM_OP_HY_STMVP: {
        Prof p(op == FVM_OP_HY_SPMV ? "hy_spmv" : "hy_stmvp", s);
        run(k_hy_spmv, bs, SZ_CELL, s, in, out, op == FVM_OP_HY_STMVP ? 1 : 0);
        break;
    }
    case FVM_OP_HY_SETMAT:
        run(k_hy_setmat, bs, SZ_MAXNF, s, in);
        break;
    default:
        break;
    }
}

void launch_hybrid_geometry(const BatchSet &bs, hipStream_t s) { run(k_hy_geom, bs, SZ_FACEI, s); }

void launch_amg_precond(const BatchSet &bs, int with_setup, hipStream_t s)
{
    const DevCase &h = *bs.host[0];
    const DevCase *dev = h.self;
    const int nl = h.amg_nl;
    auto grid = [](int n) { return dim3((unsigned)((n + kBlock - 1) / kBlock > 0 ? (n + kBlock - 1) / kBlock : 1)); };
    // the levels from l0 on (l0 >= 1, below the coarsest) run in one launch
    // when their structure fits in LDS; otherwise l0 = nl - 1
    int l0 = nl - 1;
    long tail_lds = -1;
    for (int l = 1; l <= nl - 2; ++l)
        if ((tail_lds = amg_tail_bytes(h.amg_n, h.amg_nf, l, nl)) >= 0) { l0 = l; break; }
    if (with_setup) {
        Prof p("amg_setup", s);
        for (int l = 1; l < nl; ++l)
            hipLaunchKernelGGL(k_amg_galerkin, grid(std::max(h.amg_n[l], h.amg_nf[l])), dim3(kBlock), 0, s, dev, l);
        hipLaunchKernelGGL(k_amg_cinv, dim3(1), dim3(kBlock), 0, s, dev);
        if (l0 < nl - 1) hipLaunchKernelGGL(k_amg_tail_pack, dim3(1), dim3(kAmgTailThreads), 0, s, dev, l0);
    }
    Prof p("amg_vcycle", s);
    // a wave per row on the coarse levels (level 0 keeps a thread per row)
    auto wgrid = [](int n) { return dim3((unsigned)std::max(1, (n + kRowsPerBlock - 1) / kRowsPerBlock)); };
    // the levels from l0 on (l0 >= 1, below the coarsest) run in one launch
    // when their structure fits in LDS; otherwise l0 = nl - 1
    for (int l = 0; l < l0; ++l) {
        if (l == 0) {
            run(k_amg_x0, bs, SZ_CELL, s, 0);
            run(k_amg_sell, bs, SZ_CELL, s, 0);
        } else if (h.amg_n[l] > kAmgWaveRows)
            hipLaunchKernelGGL(k_amg_down, grid(h.amg_n[l]), dim3(kBlock), 0, s, dev, l);
        else hipLaunchKernelGGL(k_amg_down_w, wgrid(h.amg_n[l]), dim3(kBlock), 0, s, dev, l);
        if (h.amg_n[l + 1] > kAmgWaveRows)
            hipLaunchKernelGGL(k_amg_restrict, grid(h.amg_n[l + 1]), dim3(kBlock), 0, s, dev, l + 1);
        else hipLaunchKernelGGL(k_amg_restrict_w, wgrid(h.amg_n[l + 1]), dim3(kBlock), 0, s, dev, l + 1);
    }
    if (l0 < nl - 1)
        hipLaunchKernelGGL(k_amg_tail, dim3(1), dim3(kAmgTailThreads), (unsigned)tail_lds, s, dev, l0, (int)tail_lds,
                           reinterpret_cast<const int4 *>(h.amg_img), h.amg_b[l0], h.amg_out[l0], h.amg_cinv,
                           h.amg_n[l0], h.amg_n[nl - 1]);
    else hipLaunchKernelGGL(k_amg_coarse, grid(h.amg_n[nl - 1]), dim3(kBlock), 0, s, dev);
    for (int l = std::min(l0, nl - 1) - 1; l >= 1; --l) {
        if (h.amg_n[l] > kAmgWaveRows) hipLaunchKernelGGL(k_amg_up, grid(h.amg_n[l]), dim3(kBlock), 0, s, dev, l);
        else hipLaunchKernelGGL(k_amg_up_w, wgrid(h.amg_n[l]), dim3(kBlock), 0, s, dev, l);
    }
    if (nl > 1) {
        run(k_amg_x0, bs, SZ_CELL, s, 1);
        run(k_amg_sell, bs, SZ_CELL, s, 1);
    } else run(k_amg_rz, bs, SZ_CELL, s);
}

void launch_clear_reduction(const BatchSet &bs, hipStream_t s) { run(k_clear_reduction, bs, SZ_CELL, s); }

// ---------------------------------------------------------------------------
// Static scratch for callers that cannot allocate (solve_pressure_static):
// the grid-reduction slots, tickets, Krylov states and a device copy of the
// case descriptor pointing at them.  Each GPU holds its own copy of the
// array at its own address, fetched once per device with that device
// current; host code uses that address, never the array's name.
// ---------------------------------------------------------------------------
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

void *static_scratch(int *hip_err)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess && (dev < 0 || dev >= 64)) e = hipErrorInvalidDevice;
    if (e != hipSuccess) {
        if (hip_err) *hip_err = (int)e;
        return nullptr;
    }
    static std::mutex mu;
    static void *ptr[64] = {};
    std::lock_guard<std::mutex> lk(mu);
    if (!ptr[dev]) {
        void *a = nullptr;
        e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !a) {
            if (hip_err) *hip_err = (int)(e != hipSuccess ? e : hipErrorInvalidSymbol);
            return nullptr;
        }
        ptr[dev] = a;
    }
    if (hip_err) *hip_err = (int)hipSuccess;
    return ptr[dev];
}
