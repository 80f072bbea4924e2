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
// Work decomposition: each block handles one contiguous chunk of cells in
// 256-wide tiles.  Block b runs on XCD b % 8; the chunk index is remapped so
// that each XCD walks one contiguous eighth of the cells, which keeps the
// neighbour gathers of a chunk in the L2 of the XCD that produced them.
//
// Reductions: a wave reduces with xor shuffles, a block through LDS, and the
// last block to finish (integer ticket) sums the per-block partials in a
// fixed order and updates the Krylov scalars in device memory.  The next
// kernels read those scalars; a solve never synchronises with the host per
// iteration, and every iteration kernel is a no-op once its system is done.
#include <hip/hip_runtime.h>

#include <cmath>

#include "fvm_internal.h"

namespace {

constexpr int kWaves = kBlock / 64;
// DIC sweeps: a NaN payload marks "not yet published"; bounded polling
constexpr unsigned long long kSentinel = 0x7FF8DEADBEEF0001ULL;   // quiet NaN with a payload
constexpr unsigned long long kQNaN = 0x7FF8000000000000ULL;
constexpr int kSpinLimit = 1 << 18;

// sentinels are written as integers: a double-typed store of a NaN constant
// need not keep its bit pattern
__device__ __forceinline__ void clear_word(double *a, int i) { reinterpret_cast<unsigned long long *>(a)[i] = kSentinel; }

__device__ __forceinline__ int logical_block()
{
    const int G = gridDim.x, b = blockIdx.x;
    return (G & 7) == 0 ? ((b & 7) * (G >> 3) + (b >> 3)) : b;
}

struct Range {
    int beg, end;
};

__device__ __forceinline__ Range block_range(int n)
{
    const int G = gridDim.x;
    long per = ((long)n + G - 1) / G;
    per = (per + kBlock - 1) / kBlock * kBlock;
    long b = (long)logical_block() * per;
    Range r;
    r.beg = (int)(b < n ? b : n);
    r.end = (int)(b + per < n ? b + per : n);
    return r;
}

template <int NV>
__device__ __forceinline__ void wave_sum(double (&v)[NV])
{
#pragma unroll
    for (int k = 0; k < NV; ++k)
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
}

// Block partial of NV sums -> per-block slot; returns true in every thread of
// the last block, with the grid totals in tot[] (LDS, valid after return).
//
// No memory fence is used (on this GPU a device-scope release writes back the
// whole L2 of the XCD).  Each block publishes its partials with device-scope
// atomic stores into slots that hold a NaN sentinel while empty, then takes
// an integer ticket.  The block that draws the last ticket reads every slot
// with device-scope atomic loads, waiting on any slot whose store has not
// landed yet, sums them in slot order and refills the slots with the
// sentinel for the next reduction.
__device__ __forceinline__ double slot_take(double *slot)
{
    unsigned long long *w = reinterpret_cast<unsigned long long *>(slot);
    unsigned long long b = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int spin = 0; b == kSentinel && spin < kSpinLimit; ++spin) {
        __builtin_amdgcn_s_sleep(1);
        b = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __hip_atomic_store(w, kSentinel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    return b == kSentinel ? __longlong_as_double((long long)kQNaN) : __longlong_as_double((long long)b);
}

__device__ __forceinline__ void slot_put(double *slot, double v)
{
    unsigned long long b = (unsigned long long)__double_as_longlong(v);
    if (b == kSentinel) b = kQNaN;
    __hip_atomic_store(reinterpret_cast<unsigned long long *>(slot), b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <int NV>
__device__ bool reduce_last(double (&v)[NV], double *partials, int stride, unsigned int *ticket, double *tot)
{
    __shared__ double lds[NV][kWaves];
    __shared__ int amlast;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    wave_sum(v);
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[k][wv] = v[k];
    __syncthreads();
    const int G = gridDim.x;
    if (threadIdx.x == 0) {
        const int lb = logical_block();
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = lds[k][0];
            for (int w = 1; w < kWaves; ++w) s += lds[k][w];
            slot_put(&partials[k * stride + lb], s);
        }
        const unsigned int t = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        amlast = (t == (unsigned int)G - 1);
    }
    __syncthreads();
    if (!amlast) return false;
    double acc[NV];
#pragma unroll
    for (int k = 0; k < NV; ++k) {
        acc[k] = 0.0;
        for (int j = threadIdx.x; j < G; j += kBlock) acc[k] += slot_take(&partials[k * stride + j]);
    }
    wave_sum(acc);
    __syncthreads();
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < NV; ++k) lds[k][wv] = acc[k];
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < NV; ++k) {
            double s = lds[k][0];
            for (int w = 1; w < kWaves; ++w) s += lds[k][w];
            tot[k] = s;
        }
        __hip_atomic_store(ticket, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    return true;
}

// y_i = diag_i x_i + sum_owned up_f x_nei + sum_nbrside lo_f x_own
__device__ __forceinline__ double row_apply(const DevCase &d, int i, const double *__restrict__ diag,
                                            const double *__restrict__ up, const double *__restrict__ lo,
                                            const double *__restrict__ x)
{
    double acc = diag[i] * x[i];
    const int f0 = d.own_start[i], f1 = d.own_start[i + 1];
    for (int f = f0; f < f1; ++f) acc += up[f] * x[d.nei[f]];
    const int k0 = d.nbr_start[i], k1 = d.nbr_start[i + 1];
    for (int k = k0; k < k1; ++k) {
        const int f = d.losort[k];
        acc += lo[f] * x[d.own[f]];
    }
    return acc;
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

// ---------------------------------------------------------------------------
// Setup and state exchange
// ---------------------------------------------------------------------------

// w = S.(C_N - Cf)/(S.d), dl = |S|^2/(S.d), k = S - dl d (internal);
// dl_b = |S|^2/(S.(Cf - C_P)) (boundary)
__global__ void k_geometry(DevCase d)
{
    const int f = blockIdx.x * kBlock + threadIdx.x;
    if (f >= d.F) return;
    const double *C = d.tmpC, *Cf = d.tmpCf;
    const int N = d.N, F = d.F;
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
__global__ void k_flux_from_U(DevCase d)
{
    const int f = blockIdx.x * kBlock + threadIdx.x;
    if (f >= d.F) return;
    const int N = d.N;
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

__global__ void k_U_in(DevCase d, const double *__restrict__ Uu)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= d.N) return;
    d.U[i] = Uu[3 * (size_t)i];
    d.U[d.N + i] = Uu[3 * (size_t)i + 1];
    d.U[2 * d.N + i] = Uu[3 * (size_t)i + 2];
}

__global__ void k_U_out(DevCase d, double *__restrict__ Uu)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= d.N) return;
    Uu[3 * (size_t)i] = d.U[i];
    Uu[3 * (size_t)i + 1] = d.U[d.N + i];
    Uu[3 * (size_t)i + 2] = d.U[2 * d.N + i];
}

__global__ void k_phi_in(DevCase d, const double *__restrict__ pu)
{
    const int f = blockIdx.x * kBlock + threadIdx.x;
    if (f >= d.F) return;
    d.phi[f] = f < d.Fi ? (double)d.face_sign[f] * pu[d.face_user[f]] : pu[f];
}

__global__ void k_phi_out(DevCase d, double *__restrict__ pu)
{
    const int f = blockIdx.x * kBlock + threadIdx.x;
    if (f >= d.F) return;
    if (f < d.Fi) pu[d.face_user[f]] = (double)d.face_sign[f] * d.phi[f];
    else pu[f] = d.phi[f];
}

// caller face order -> canonical order (orientation-free face values)
__global__ void k_gather_faces(DevCase d, const double *__restrict__ uv, double *__restrict__ out)
{
    const int f = blockIdx.x * kBlock + threadIdx.x;
    if (f >= d.F) return;
    out[f] = f < d.Fi ? uv[d.face_user[f]] : uv[f];
}

// ---------------------------------------------------------------------------
// Momentum assembly
// ---------------------------------------------------------------------------

// Gauss gradient of a cell scalar x with the boundary rule of `kinds`/`vals`
// (FIXED value, ZERO_GRAD owner value, EMPTY skipped); returns sum S phi_f
// (not divided by V)
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

// gradU[3c + k][i] = d U_c / d x_k (start-of-step U; non-orthogonal meshes)
__global__ void k_gradU(DevCase d)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= d.N) return;
    const int N = d.N;
    for (int c = 0; c < 3; ++c) {
        double g0, g1, g2;
        gauss_sum(d, i, d.U + (size_t)c * N, d.patch_uk, d.patch_uv + c, 3, g0, g1, g2);
        const double V = d.V[i];
        d.gradU[(size_t)(3 * c) * N + i] = g0 / V;
        d.gradU[(size_t)(3 * c + 1) * N + i] = g1 / V;
        d.gradU[(size_t)(3 * c + 2) * N + i] = g2 / V;
    }
}

// upper = F(1-w) - nu dl, lower = -F w - nu dl; non-orthogonal source
// ns_c = nu k.(w gradU_c,P + (1-w) gradU_c,N)
__global__ void k_mom_face(DevCase d, double nu, int upwind)
{
    const int f = blockIdx.x * kBlock + threadIdx.x;
    if (f >= d.Fi) return;
    const double Fl = d.phi[f];
    const double w = upwind ? (Fl >= 0.0 ? 1.0 : 0.0) : d.w[f];
    const double D = nu * d.dl[f];
    d.upper[f] = Fl * (1.0 - w) - D;
    d.lower[f] = -Fl * w - D;
    if (d.nonorth) {
        const int N = d.N, P = d.own[f], Q = d.nei[f];
        const double wi = d.w[f];
        const double k0 = d.kx[f], k1 = d.ky[f], k2 = d.kz[f];
        for (int c = 0; c < 3; ++c) {
            const double *g = d.gradU + (size_t)(3 * c) * N;
            const double a0 = wi * g[P] + (1.0 - wi) * g[Q];
            const double a1 = wi * g[N + P] + (1.0 - wi) * g[N + Q];
            const double a2 = wi * g[2 * N + P] + (1.0 - wi) * g[2 * N + Q];
            d.ns[(size_t)c * d.Fi + f] = nu * (k0 * a0 + k1 * a1 + k2 * a2);
        }
    }
}

// diag, src (without the pressure gradient) and rhs = src - V grad p.
// dt > 0: transient term V/dt, V U/dt.  alpha_u < 1: implicit relaxation
// diag <- diag/alpha, src += (1-alpha)/alpha diag_orig U.
__global__ void k_mom_cell(DevCase d, double nu, double dt, double alpha_u, int upwind)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= d.N) return;
    const int N = d.N;
    const double V = d.V[i];
    const double U0 = d.U[i], U1 = d.U[N + i], U2 = d.U[2 * N + i];
    double dg = 0.0, s0 = 0.0, s1 = 0.0, s2 = 0.0;
    if (dt > 0.0) {
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
            s0 += d.ns[f]; s1 += d.ns[(size_t)d.Fi + f]; s2 += d.ns[2 * (size_t)d.Fi + f];
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
            s0 -= d.ns[f]; s1 -= d.ns[(size_t)d.Fi + f]; s2 -= d.ns[2 * (size_t)d.Fi + f];
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
    if (alpha_u < 1.0) {
        const double d0 = dg;
        dg = d0 / alpha_u;
        const double c = (1.0 - alpha_u) / alpha_u * d0;
        s0 += c * U0; s1 += c * U1; s2 += c * U2;
    }
    d.mdiag[i] = dg;
    d.src[i] = s0; d.src[N + i] = s1; d.src[2 * N + i] = s2;
    d.rhs[i] = s0 - V * (g0 / V);
    d.rhs[N + i] = s1 - V * (g1 / V);
    d.rhs[2 * N + i] = s2 - V * (g2 / V);
}

// ---------------------------------------------------------------------------
// Pressure corrector
// ---------------------------------------------------------------------------

// H = src - sum a_PN U_N, rAU = V/a_PP, HbyA = H/a_PP; optional grad p
__global__ void k_hbya(DevCase d, int with_gradp)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= d.N) return;
    const int N = d.N;
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
    if (with_gradp) {
        double g0, g1, g2;
        gauss_sum(d, i, d.p, d.patch_pk, d.patch_pv, 1, g0, g1, g2);
        const double V = d.V[i];
        d.gradp[i] = g0 / V; d.gradp[N + i] = g1 / V; d.gradp[2 * N + i] = g2 / V;
    }
}

__global__ void k_gradp(DevCase d)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= d.N) return;
    double g0, g1, g2;
    gauss_sum(d, i, d.p, d.patch_pk, d.patch_pv, 1, g0, g1, g2);
    const double V = d.V[i];
    d.gradp[i] = g0 / V; d.gradp[d.N + i] = g1 / V; d.gradp[2 * d.N + i] = g2 / V;
}

// face pass: phiH = S.interp(HbyA) (boundary per U kind), gam = interp(rAU)
// (boundary rAU_P), poff = -gam dl, tno = gam k.interp(grad p)
__global__ void k_p_face(DevCase d)
{
    const int f = blockIdx.x * kBlock + threadIdx.x;
    if (f >= d.F) return;
    const int N = d.N;
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

// cell pass: pdiag, pb (divergence, fixed-p terms, non-orthogonal part), pin
__global__ void k_p_cell(DevCase d, double p_ref, int with_div)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= d.N) return;
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
        b += a * p_ref;
    }
    d.pdiag[i] = dg;
    if (with_div) d.pb[i] = b;
    else d.pb[i] += b;
}

// gamma given per face (canonical order) -> poff, gam
__global__ void k_p_face_gamma(DevCase d, const double *__restrict__ gam)
{
    const int f = blockIdx.x * kBlock + threadIdx.x;
    if (f >= d.F) return;
    const double g = gam[f];
    d.gam[f] = g;
    if (f < d.Fi) d.poff[f] = -(g * d.dl[f]);
}

// phi = phiH - g (p_N - p_P) - tno (internal); p FIXED: phiH - g_b (p_b - p_P)
__global__ void k_flux_corr(DevCase d)
{
    const int f = blockIdx.x * kBlock + threadIdx.x;
    if (f >= d.F) return;
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

__global__ void k_p_relax(DevCase d, double alpha_p)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= d.N) return;
    d.p[i] = d.p_prev[i] + alpha_p * (d.p[i] - d.p_prev[i]);
}

// U = HbyA - rAU grad p (new p)
__global__ void k_U_corr(DevCase d)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= d.N) return;
    const int N = d.N;
    double g0, g1, g2;
    gauss_sum(d, i, d.p, d.patch_pk, d.patch_pv, 1, g0, g1, g2);
    const double V = d.V[i], r = d.rAU[i];
    d.U[i] = d.HbyA[i] - r * (g0 / V);
    d.U[N + i] = d.HbyA[N + i] - r * (g1 / V);
    d.U[2 * N + i] = d.HbyA[2 * N + i] - r * (g2 / V);
}

// ---------------------------------------------------------------------------
// Krylov solvers (Barrett et al., "Templates": CG and BiCG)
//
// The iteration kernels are templated on the vector/matrix value type: the
// FP64 solves and the FP32 inner solves of the mixed-precision refinement run
// the same code over different arrays.  Every dot product and residual sum is
// accumulated in FP64 whatever the vector type.
// ---------------------------------------------------------------------------

__device__ __forceinline__ void set_done(KState &s, int status)
{
    s.status = status;
    s.done = 1;
}

template <class T>
__device__ __forceinline__ T row_apply_t(const DevCase &d, int i, const T *__restrict__ diag, const T *__restrict__ up,
                                         const T *__restrict__ lo, const T *__restrict__ x)
{
    T acc = diag[i] * x[i];
    const int f0 = d.own_start[i], f1 = d.own_start[i + 1];
    for (int f = f0; f < f1; ++f) acc += up[f] * x[d.nei[f]];
    const int k0 = d.nbr_start[i], k1 = d.nbr_start[i + 1];
    for (int k = k0; k < k1; ++k) {
        const int f = d.losort[k];
        acc += lo[f] * x[d.own[f]];
    }
    return acc;
}

// symmetric system (pressure): one coefficient per face
template <class T>
struct CGView {
    const T *diag, *off;
    T *x, *r, *p, *q;
    const double *z;    // DIC output (FP64 path), else nullptr
    KState *ks;
};

// non-symmetric system (momentum), three right-hand sides sharing A
template <class T>
struct BiView {
    const T *diag, *up, *lo;
    T *x, *r, *rt, *p, *pt, *q, *qt;     // [3][N]
    KState *ks;                          // [3]
};

// ---- BiCG --------------------------------------------------------------

// p = z + beta p, p~ = z~ + beta p~ (z = r/diag, z~ = r~/diag)
template <class T>
__global__ void k_bicg_dir(DevCase d, BiView<T> v)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= d.N) return;
    const int N = d.N;
    const T dg = v.diag[i];
    for (int c = 0; c < 3; ++c) {
        const KState &s = v.ks[c];
        if (s.done) continue;
        const size_t j = (size_t)c * N + i;
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
__global__ void __launch_bounds__(kBlock) k_bicg_spmv(DevCase d, BiView<T> v)
{
    int act[3];
    for (int c = 0; c < 3; ++c) act[c] = !v.ks[c].done;
    if (!act[0] && !act[1] && !act[2]) return;
    const Range rg = block_range(d.N);
    const int N = d.N;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int i = rg.beg + threadIdx.x; i < rg.end; i += kBlock) {
        for (int c = 0; c < 3; ++c) {
            if (!act[c]) continue;
            const T *p = v.p + (size_t)c * N, *pt = v.pt + (size_t)c * N;
            const T q = row_apply_t<T>(d, i, v.diag, v.up, v.lo, p);
            const T qt = row_apply_t<T>(d, i, v.diag, v.lo, v.up, pt);
            v.q[(size_t)c * N + i] = q;
            v.qt[(size_t)c * N + i] = qt;
            acc[c] += (double)pt[i] * (double)q;
        }
    }
    __shared__ double tot[3];
    if (reduce_last<3>(acc, d.partials, d.red_stride, d.ticket, tot) && threadIdx.x == 0) {
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
__global__ void __launch_bounds__(kBlock) k_bicg_update(DevCase d, BiView<T> v)
{
    int act[3];
    T al[3];
    for (int c = 0; c < 3; ++c) { act[c] = !v.ks[c].done; al[c] = (T)v.ks[c].alpha; }
    if (!act[0] && !act[1] && !act[2]) return;
    const Range rg = block_range(d.N);
    const int N = d.N;
    double acc[6] = {0, 0, 0, 0, 0, 0};
    for (int i = rg.beg + threadIdx.x; i < rg.end; i += kBlock) {
        const T dg = v.diag[i];
        for (int c = 0; c < 3; ++c) {
            if (!act[c]) continue;
            const size_t j = (size_t)c * N + i;
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
    if (reduce_last<6>(acc, d.partials, d.red_stride, d.ticket, tot) && threadIdx.x == 0) {
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
__global__ void __launch_bounds__(kBlock) k_bicg_sumx(DevCase d)
{
    const Range r = block_range(d.N);
    const int N = d.N;
    double v[3] = {0.0, 0.0, 0.0};
    for (int i = r.beg + threadIdx.x; i < r.end; i += kBlock)
        for (int c = 0; c < 3; ++c) v[c] += d.U[(size_t)c * N + i];
    __shared__ double tot[3];
    if (reduce_last<3>(v, d.partials, d.red_stride, d.ticket, tot) && threadIdx.x == 0)
        for (int c = 0; c < 3; ++c) d.ks[c].xbar = tot[c] / (double)N;
}

// FP64 start: r = b - A x, r~ = r, normalisation, first rho = z.r~
__global__ void __launch_bounds__(kBlock) k_bicg_init(DevCase d)
{
    const Range rg = block_range(d.N);
    const int N = d.N;
    double xb[3];
    for (int c = 0; c < 3; ++c) xb[c] = d.ks[c].xbar;
    double v[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};   // nf_c, |r|_c, rho_c
    for (int i = rg.beg + threadIdx.x; i < rg.end; i += kBlock) {
        const double a1 = row_sum(d, i, d.mdiag, d.upper, d.lower);
        const double dg = d.mdiag[i];
        for (int c = 0; c < 3; ++c) {
            const double *x = d.U + (size_t)c * N;
            const double ax = row_apply(d, i, d.mdiag, d.upper, d.lower, x);
            const double b = d.rhs[(size_t)c * N + i];
            const double r = b - ax;
            d.r[(size_t)c * N + i] = r;
            d.rt[(size_t)c * N + i] = r;
            v[c] += fabs(ax - xb[c] * a1) + fabs(b - xb[c] * a1);
            v[3 + c] += fabs(r);
            const double z = r / dg;
            v[6 + c] += z * r;
        }
    }
    __shared__ double tot[9];
    if (reduce_last<9>(v, d.partials, d.red_stride, d.ticket, tot) && threadIdx.x == 0) {
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
            if (!isfinite(s.nres0)) set_done(s, FVM_ENUMERIC);
            else if (s.nres0 <= s.tol_eff) set_done(s, FVM_OK);
            else if (tot[6 + c] == 0.0 || !isfinite(tot[6 + c])) { set_done(s, FVM_ENUMERIC); s.iters = 1; }
            else s.rho = tot[6 + c];
        }
    }
}

// ---- CG ----------------------------------------------------------------

// p = z + beta p (Jacobi z = r/diag; DIC z from the sweeps)
template <class T>
__global__ void k_cg_dir(DevCase d, CGView<T> v)
{
    const KState &s = *v.ks;
    if (s.done) return;
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= d.N) return;
    const T z = v.z ? (T)v.z[i] : v.r[i] / v.diag[i];
    v.p[i] = s.first ? z : z + (T)s.beta * v.p[i];
}

// q = A p, p.q -> alpha
template <class T>
__global__ void __launch_bounds__(kBlock) k_cg_spmv(DevCase d, CGView<T> v)
{
    if (v.ks->done) return;
    const Range rg = block_range(d.N);
    double acc[1] = {0.0};
    for (int i = rg.beg + threadIdx.x; i < rg.end; i += kBlock) {
        const T q = row_apply_t<T>(d, i, v.diag, v.off, v.off, v.p);
        v.q[i] = q;
        acc[0] += (double)v.p[i] * (double)q;
    }
    __shared__ double tot[1];
    if (reduce_last<1>(acc, d.partials, d.red_stride, d.ticket, tot) && threadIdx.x == 0) {
        KState &s = *v.ks;
        if (!(tot[0] > 0.0) || !isfinite(tot[0])) { set_done(s, FVM_ENUMERIC); s.iters += 1; }
        else s.alpha = s.rho / tot[0];
    }
}

// x += alpha p, r -= alpha q, |r| -> stop test; Jacobi: rho = r.(r/diag), beta
template <class T>
__global__ void __launch_bounds__(kBlock) k_cg_update(DevCase d, CGView<T> v, int dic)
{
    if (v.ks->done) return;
    const T al = (T)v.ks->alpha;
    const Range rg = block_range(d.N);
    double acc[2] = {0.0, 0.0};
    for (int i = rg.beg + threadIdx.x; i < rg.end; i += kBlock) {
        v.x[i] += al * v.p[i];
        const T r = v.r[i] - al * v.q[i];
        v.r[i] = r;
        acc[0] += fabs((double)r);
        if (!dic) acc[1] += (double)r * (double)(r / v.diag[i]);
    }
    __shared__ double tot[2];
    if (reduce_last<2>(acc, d.partials, d.red_stride, d.ticket, tot) && threadIdx.x == 0) {
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

__global__ void __launch_bounds__(kBlock) k_pcg_sumx(DevCase d)
{
    const Range r = block_range(d.N);
    double v[1] = {0.0};
    for (int i = r.beg + threadIdx.x; i < r.end; i += kBlock) v[0] += d.p[i];
    __shared__ double tot[1];
    if (reduce_last<1>(v, d.partials, d.red_stride, d.ticket, tot) && threadIdx.x == 0)
        d.ks[3].xbar = tot[0] / (double)d.N;
}

// FP64 start: r = b - A x; normalisation; Jacobi: first rho = r.(r/diag)
__global__ void __launch_bounds__(kBlock) k_pcg_init(DevCase d, int dic)
{
    const Range rg = block_range(d.N);
    const double xb = d.ks[3].xbar;
    double v[3] = {0.0, 0.0, 0.0};
    for (int i = rg.beg + threadIdx.x; i < rg.end; i += kBlock) {
        const double a1 = row_sum(d, i, d.pdiag, d.poff, d.poff);
        const double ax = row_apply(d, i, d.pdiag, d.poff, d.poff, d.p);
        const double b = d.pb[i];
        const double r = b - ax;
        d.r[i] = r;
        v[0] += fabs(ax - xb * a1) + fabs(b - xb * a1);
        v[1] += fabs(r);
        if (!dic) v[2] += r * (r / d.pdiag[i]);
        else {
            clear_word(d.dstar, i);
            clear_word(d.y, i);
            clear_word(d.z, i);
        }
    }
    __shared__ double tot[3];
    if (reduce_last<3>(v, d.partials, d.red_stride, d.ticket, tot) && threadIdx.x == 0) {
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
// Mixed precision: FP64 iterative refinement around FP32 inner solves
//
// Outer (FP64, states ks[0..3]):  r = b - A x  ->  if nres <= tol: stop
//   inner (FP32, states ks[4..7]): A e = s r from e = 0 to a relative
//                                  reduction eta, s = N / sum|r| (keeps the
//                                  demoted residual O(1))
//   x += e / s  (FP64).
// The outer iteration count is the total number of inner iterations.
// ---------------------------------------------------------------------------

// FP32 copies of the assembled matrix values (the topology is shared)
__global__ void k_mx_cvt(DevCase d, int kind)
{
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (kind == 1) {
        if (t < d.N) d.f_pdiag[t] = (float)d.pdiag[t];
        if (t < d.Fi) d.f_poff[t] = (float)d.poff[t];
    } else {
        if (t < d.N) d.f_diag[t] = (float)d.mdiag[t];
        if (t < d.Fi) { d.f_up[t] = (float)d.upper[t]; d.f_lo[t] = (float)d.lower[t]; }
    }
}

__device__ __forceinline__ double mx_scale(const KState &o, int N) { return (double)N / (o.nres * o.nf); }

// inner start: r_in = s r (FP32), e = 0, inner normalisation sum|r_in|,
// Jacobi rho.  kind 1: pressure (one system), kind 0: momentum (three).
__global__ void __launch_bounds__(kBlock) k_mx_inner_init(DevCase d, int kind)
{
    const int nsys = kind == 1 ? 1 : 3, o0 = kind == 1 ? 3 : 0, i0 = kind == 1 ? 7 : 4;
    int act[3];
    double sc[3];
    for (int c = 0; c < 3; ++c) {
        act[c] = c < nsys && !d.ks[o0 + c].done;
        sc[c] = act[c] ? mx_scale(d.ks[o0 + c], d.N) : 0.0;
    }
    if (!act[0] && !act[1] && !act[2]) return;
    const Range rg = block_range(d.N);
    const int N = d.N;
    const float *diag = kind == 1 ? d.f_pdiag : d.f_diag;
    double v[6] = {0, 0, 0, 0, 0, 0};
    for (int i = rg.beg + threadIdx.x; i < rg.end; i += kBlock) {
        const float dg = diag[i];
        for (int c = 0; c < nsys; ++c) {
            if (!act[c]) continue;
            const size_t j = (size_t)c * N + i;
            const float r = (float)(sc[c] * d.r[j]);
            d.f_r[j] = r;
            d.f_x[j] = 0.0f;
            if (kind == 0) d.f_rt[j] = r;
            v[c] += fabs((double)r);
            v[3 + c] += (double)(r / dg) * (double)r;
        }
    }
    __shared__ double tot[6];
    if (reduce_last<6>(v, d.partials, d.red_stride, d.ticket, tot) && threadIdx.x == 0) {
        for (int c = 0; c < nsys; ++c) {
            KState &s = d.ks[i0 + c];
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
            const bool bad = kind == 1 ? !(tot[3 + c] > 0.0) : tot[3 + c] == 0.0;
            if (!isfinite(tot[c]) || !(tot[c] > 0.0)) set_done(s, FVM_ENUMERIC);
            else if (bad || !isfinite(tot[3 + c])) { set_done(s, FVM_ENUMERIC); s.iters = 1; }
            else s.rho = tot[3 + c];
        }
    }
}

// x += e / s (FP64), for the systems whose outer loop is still running
__global__ void k_mx_correct(DevCase d, int kind)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= d.N) return;
    const int nsys = kind == 1 ? 1 : 3, o0 = kind == 1 ? 3 : 0;
    double *x = kind == 1 ? d.p : d.U;
    for (int c = 0; c < nsys; ++c) {
        const KState &o = d.ks[o0 + c];
        if (o.done) continue;
        const double s = mx_scale(o, d.N);
        const size_t j = (size_t)c * d.N + i;
        x[j] += (double)d.f_x[j] / s;
    }
}

// outer residual after a correction: r = b - A x (FP64), nres, stop test;
// the inner iterations are added to the outer count
__global__ void __launch_bounds__(kBlock) k_mx_resid(DevCase d, int kind)
{
    const int nsys = kind == 1 ? 1 : 3, o0 = kind == 1 ? 3 : 0, i0 = kind == 1 ? 7 : 4;
    int act[3];
    for (int c = 0; c < 3; ++c) act[c] = c < nsys && !d.ks[o0 + c].done;
    if (!act[0] && !act[1] && !act[2]) return;
    const Range rg = block_range(d.N);
    const int N = d.N;
    const double *diag = kind == 1 ? d.pdiag : d.mdiag;
    const double *up = kind == 1 ? d.poff : d.upper;
    const double *lo = kind == 1 ? d.poff : d.lower;
    const double *xb = kind == 1 ? d.p : d.U;
    const double *bb = kind == 1 ? d.pb : d.rhs;
    double v[3] = {0, 0, 0};
    for (int i = rg.beg + threadIdx.x; i < rg.end; i += kBlock) {
        for (int c = 0; c < nsys; ++c) {
            if (!act[c]) continue;
            const size_t j = (size_t)c * N + i;
            const double r = bb[j] - row_apply(d, i, diag, up, lo, xb + (size_t)c * N);
            d.r[j] = r;
            v[c] += fabs(r);
        }
    }
    __shared__ double tot[3];
    if (reduce_last<3>(v, d.partials, d.red_stride, d.ticket, tot) && threadIdx.x == 0) {
        for (int c = 0; c < nsys; ++c) {
            if (!act[c]) continue;
            KState &o = d.ks[o0 + c];
            const KState &in = d.ks[i0 + c];
            o.iters += in.iters;
            o.nres = tot[c] / o.nf;
            if (in.status == FVM_ENUMERIC || !isfinite(o.nres)) set_done(o, FVM_ENUMERIC);
            else if (o.nres <= o.tol_eff) set_done(o, FVM_OK);
            else if (o.iters >= o.max_iter) set_done(o, FVM_WARN_MAXITER);
        }
    }
}

// ---------------------------------------------------------------------------
// DIC triangular sweeps, sync-free in level order
//
// The diagonal-only incomplete Cholesky factor D* and the two triangular
// solves of M = (D* + L) D*^-1 (D* + U) are recurrences over the lower
// (upper) neighbours of each cell.  Cells are processed in the order of the
// dependency levels computed at mesh ingest; tiles of 256 cells are claimed
// through an atomic ticket, so every dependency of a tile lies in a tile that
// has already been claimed by a running or finished block.  A value is
// published with one 64-bit device-scope store into an array pre-filled with
// a NaN sentinel: the value is its own ready flag, so no fence is needed and
// a reader polls exactly the word it consumes.  Each lane keeps consuming
// dependencies as they appear (no lane waits inside a loop another lane of
// its wave must leave first), and polling is bounded: past the limit the
// value is published as NaN, which the solver reports as a breakdown instead
// of hanging.  Per cell the sums run over neighbours in ascending index.
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool dic_try(const double *a, int j, double &v)
{
    const unsigned long long b =
        __hip_atomic_load(reinterpret_cast<const unsigned long long *>(a + j), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (b == kSentinel) return false;
    v = __longlong_as_double((long long)b);
    return true;
}

__device__ __forceinline__ void dic_put(double *a, int i, double v)
{
    unsigned long long b = (unsigned long long)__double_as_longlong(v);
    if (b == kSentinel) b = kQNaN;
    __hip_atomic_store(reinterpret_cast<unsigned long long *>(a + i), b, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// MODE 0: D*_i = A_ii - sum_{j<i} a_ij^2 / D*_j
// MODE 1: y_i = (r_i - sum_{j<i} a_ij y_j) / D*_i      (also clears z)
// MODE 2: z_i = y_i - (sum_{j>i} a_ij z_j) / D*_i      (reverse order; r.z)
//
// A cell's dependency list (neighbour index and coefficient) is read into
// registers before polling, so each poll round is one batch of independent
// device-scope loads of the values still missing; once all are present the
// sum is formed in ascending neighbour order.  Cells with more than kDicDeps
// dependencies take a streaming path that consumes them one at a time.
constexpr int kDicDeps = 8;

template <int MODE>
__global__ void __launch_bounds__(kBlock) k_dic_sweep(DevCase d)
{
    if (d.ks[3].done) return;
    __shared__ int tile;
    if (threadIdx.x == 0) tile = (int)atomicAdd(&d.ticket[1], 1u);
    __syncthreads();
    const int n = d.N;
    const int pos = tile * kBlock + threadIdx.x;
    const bool live = pos < n;
    const int i = live ? (MODE == 2 ? d.lvl_cells[n - 1 - pos] : d.lvl_cells[pos]) : 0;
    int k0, k1;
    double acc;
    const double *src;
    if (MODE == 2) { k0 = d.own_start[i]; k1 = d.own_start[i + 1]; acc = 0.0; src = d.z; }
    else { k0 = d.nbr_start[i]; k1 = d.nbr_start[i + 1]; acc = MODE == 0 ? d.pdiag[i] : d.r[i]; src = MODE == 0 ? d.dstar : d.y; }
    if (!live) k1 = k0;
    const int nd = k1 - k0;
    const bool fast = nd <= kDicDeps;
    int js[kDicDeps];
    double as[kDicDeps], vs[kDicDeps];
#pragma unroll
    for (int t = 0; t < kDicDeps; ++t) {
        js[t] = 0; as[t] = 0.0; vs[t] = 0.0;
        if (fast && t < nd) {
            const int f = MODE == 2 ? k0 + t : d.losort[k0 + t];
            js[t] = MODE == 2 ? d.nei[f] : d.own[f];
            as[t] = d.poff[f];
        }
    }
    const double dsi = (MODE != 0 && live) ? d.dstar[i] : 1.0;
    const double yi = (MODE == 2 && live) ? d.y[i] : 0.0;
    unsigned int missing = fast ? (nd >= 32 ? 0xffffffffu : ((1u << nd) - 1u)) : 0u;
    int k = k0;               // streaming path cursor
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
#pragma unroll
                for (int t = 0; t < kDicDeps; ++t) {
                    if (missing & (1u << t)) {
                        double v;
                        if (dic_try(src, js[t], v)) { vs[t] = v; missing &= ~(1u << t); }
                    }
                }
                ready = missing == 0u;
                if (ready) {
#pragma unroll
                    for (int t = 0; t < kDicDeps; ++t) {
                        if (t < nd) {
                            if (MODE == 0) acc -= as[t] * as[t] / vs[t];
                            else if (MODE == 1) acc -= as[t] * vs[t];
                            else acc += as[t] * vs[t];
                        }
                    }
                }
            } else {
                ready = true;
                while (k < k1) {
                    const int f = MODE == 2 ? k : d.losort[k];
                    const int j = MODE == 2 ? d.nei[f] : d.own[f];
                    double v;
                    if (!dic_try(src, j, v)) { ready = false; break; }
                    const double a = d.poff[f];
                    if (MODE == 0) acc -= a * a / v;
                    else if (MODE == 1) acc -= a * v;
                    else acc += a * v;
                    ++k;
                }
            }
            if (ready) {
                if (MODE == 0) dic_put(d.dstar, i, acc);
                else if (MODE == 1) { dic_put(d.y, i, acc / dsi); clear_word(d.z, i); }
                else {
                    const double zi = yi - acc / dsi;
                    dic_put(d.z, i, zi);
                    clear_word(d.y, i);
                    part = d.r[i] * zi;
                }
                fin = true;
            } else if (++spins > kSpinLimit) {
                dic_put(MODE == 0 ? d.dstar : (MODE == 1 ? d.y : d.z), i, __longlong_as_double((long long)kQNaN));
                if (MODE == 2) part = __longlong_as_double((long long)kQNaN);
                d.ticket[8] = 1u;
                fin = true;
            }
        }
        if (__all(fin)) break;
        __builtin_amdgcn_s_sleep(1);
    }
    if (MODE == 2) {
        double v[1] = {part};
        __shared__ double tot[1];
        if (reduce_last<1>(v, d.partials, d.red_stride, d.ticket, tot) && threadIdx.x == 0) {
            KState &s = d.ks[3];
            __hip_atomic_store(&d.ticket[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
            if (t == gridDim.x - 1) {
                __hip_atomic_store(&d.ticket[1], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&d.ticket[2], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
        }
    }
}

__global__ void k_fill_sentinel(double *a, long n)
{
    const long i = (long)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) clear_word(a, (int)i);
}

__global__ void k_dic_reset(DevCase d)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i == 0) {
        d.ks[3].done = 0;
        d.ks[3].iters = 0;
        d.ks[3].status = FVM_OK;
    }
    if (i >= d.N) return;
    clear_word(d.dstar, i);
    clear_word(d.y, i);
    clear_word(d.z, i);
}

__global__ void k_set_ctl(KState *ks, int first, int count, double tol, double rel_tol, int max_iter)
{
    const int k = threadIdx.x;
    if (k >= count) return;
    ks[first + k].tol = tol;
    ks[first + k].rel_tol = rel_tol;
    ks[first + k].max_iter = max_iter;
}

__global__ void k_set_patch(DevCase d, int pt, double u0, double u1, double u2, double pv)
{
    if (threadIdx.x != 0) return;
    d.patch_uv[3 * pt] = u0;
    d.patch_uv[3 * pt + 1] = u1;
    d.patch_uv[3 * pt + 2] = u2;
    d.patch_pv[pt] = pv;
}

inline int cdiv(long a, long b) { return (int)((a + b - 1) / b); }

}  // namespace

// ---------------------------------------------------------------------------
// Launchers
// ---------------------------------------------------------------------------

int grid_for(int n)
{
    int g = cdiv(n, kBlock);
    if (g > kMaxGrid) g = kMaxGrid;
    if (g >= 8) g = g / 8 * 8;
    return g < 1 ? 1 : g;
}

#define LAUNCH_N(kern, n, s, ...)                                                             \
    do {                                                                                      \
        if ((n) > 0) hipLaunchKernelGGL(kern, dim3(cdiv((n), kBlock)), dim3(kBlock), 0, s, __VA_ARGS__); \
    } while (0)
#define LAUNCH_R(kern, n, s, ...) hipLaunchKernelGGL(kern, dim3(grid_for(n)), dim3(kBlock), 0, s, __VA_ARGS__)

void launch_geometry(const DevCase &d, hipStream_t s) { LAUNCH_N(k_geometry, d.F, s, d); }
void launch_flux_from_U(const DevCase &d, hipStream_t s) { LAUNCH_N(k_flux_from_U, d.F, s, d); }
void launch_U_in(const DevCase &d, const double *U, hipStream_t s) { LAUNCH_N(k_U_in, d.N, s, d, U); }
void launch_U_out(const DevCase &d, double *U, hipStream_t s) { LAUNCH_N(k_U_out, d.N, s, d, U); }
void launch_phi_in(const DevCase &d, const double *phi, hipStream_t s) { LAUNCH_N(k_phi_in, d.F, s, d, phi); }
void launch_phi_out(const DevCase &d, double *phi, hipStream_t s) { LAUNCH_N(k_phi_out, d.F, s, d, phi); }
void launch_gather_faces(const DevCase &d, const double *uv, double *out, hipStream_t s)
{
    LAUNCH_N(k_gather_faces, d.F, s, d, uv, out);
}

void launch_gradU(const DevCase &d, hipStream_t s) { LAUNCH_N(k_gradU, d.N, s, d); }
void launch_mom_face(const DevCase &d, double nu, int upwind, hipStream_t s)
{
    prof_begin("mom_face", s);
    LAUNCH_N(k_mom_face, d.Fi, s, d, nu, upwind);
    prof_end("mom_face", s);
}
void launch_mom_cell(const DevCase &d, double nu, double dt, double alpha_u, int upwind, hipStream_t s)
{
    prof_begin("mom_cell", s);
    LAUNCH_N(k_mom_cell, d.N, s, d, nu, dt, alpha_u, upwind);
    prof_end("mom_cell", s);
}
void launch_hbya(const DevCase &d, int with_gradp, hipStream_t s)
{
    prof_begin("hbya", s);
    LAUNCH_N(k_hbya, d.N, s, d, with_gradp);
    prof_end("hbya", s);
}
void launch_gradp(const DevCase &d, hipStream_t s) { LAUNCH_N(k_gradp, d.N, s, d); }
void launch_p_face(const DevCase &d, hipStream_t s)
{
    prof_begin("p_face", s);
    LAUNCH_N(k_p_face, d.F, s, d);
    prof_end("p_face", s);
}
void launch_p_cell(const DevCase &d, double p_ref, hipStream_t s)
{
    prof_begin("p_cell", s);
    LAUNCH_N(k_p_cell, d.N, s, d, p_ref, 1);
    prof_end("p_cell", s);
}
void launch_p_system_from_gamma(const DevCase &d, const double *gam, const double *rhs, double p_ref, hipStream_t s)
{
    LAUNCH_N(k_p_face_gamma, d.F, s, d, gam);
    (void)hipMemcpyAsync(d.pb, rhs, sizeof(double) * (size_t)d.N, hipMemcpyDeviceToDevice, s);
    LAUNCH_N(k_p_cell, d.N, s, d, p_ref, 0);
}
void launch_flux_corr(const DevCase &d, hipStream_t s)
{
    prof_begin("flux_corr", s);
    LAUNCH_N(k_flux_corr, d.F, s, d);
    prof_end("flux_corr", s);
}
void launch_p_relax(const DevCase &d, double alpha_p, hipStream_t s) { LAUNCH_N(k_p_relax, d.N, s, d, alpha_p); }
void launch_U_corr(const DevCase &d, hipStream_t s)
{
    prof_begin("U_corr", s);
    LAUNCH_N(k_U_corr, d.N, s, d);
    prof_end("U_corr", s);
}

void launch_bicg_init(const DevCase &d, hipStream_t s)
{
    LAUNCH_R(k_bicg_sumx, d.N, s, d);
    LAUNCH_R(k_bicg_init, d.N, s, d);
}

static BiView<double> bi64(const DevCase &d)
{
    return BiView<double>{d.mdiag, d.upper, d.lower, d.U, d.r, d.rt, d.pp, d.pt, d.q, d.qt, d.ks};
}

static BiView<float> bi32(const DevCase &d)
{
    return BiView<float>{d.f_diag, d.f_up, d.f_lo, d.f_x, d.f_r, d.f_rt, d.f_p, d.f_pt, d.f_q, d.f_qt, d.ks + 4};
}

static CGView<double> cg64(const DevCase &d, int dic)
{
    return CGView<double>{d.pdiag, d.poff, d.p, d.r, d.pp, d.q, dic ? d.z : nullptr, d.ks + 3};
}

static CGView<float> cg32(const DevCase &d)
{
    return CGView<float>{d.f_pdiag, d.f_poff, d.f_x, d.f_r, d.f_p, d.f_q, nullptr, d.ks + 7};
}

void launch_bicg_iter(const DevCase &d, hipStream_t s)
{
    const BiView<double> v = bi64(d);
    LAUNCH_N(k_bicg_dir<double>, d.N, s, d, v);
    prof_begin("bicg_spmv", s);
    LAUNCH_R(k_bicg_spmv<double>, d.N, s, d, v);
    prof_end("bicg_spmv", s);
    LAUNCH_R(k_bicg_update<double>, d.N, s, d, v);
}

void launch_pcg_init(const DevCase &d, int dic, hipStream_t s)
{
    LAUNCH_R(k_pcg_sumx, d.N, s, d);
    LAUNCH_R(k_pcg_init, d.N, s, d, dic);
}

void launch_mx_cvt(const DevCase &d, int kind, hipStream_t s)
{
    LAUNCH_N(k_mx_cvt, d.N > d.Fi ? d.N : d.Fi, s, d, kind);
}

void launch_mx_inner_init(const DevCase &d, int kind, hipStream_t s) { LAUNCH_R(k_mx_inner_init, d.N, s, d, kind); }

void launch_mx_inner_iter(const DevCase &d, int kind, hipStream_t s)
{
    if (kind == 1) {
        const CGView<float> v = cg32(d);
        prof_begin("pcg32_dir", s);
        LAUNCH_N(k_cg_dir<float>, d.N, s, d, v);
        prof_end("pcg32_dir", s);
        prof_begin("pcg32_spmv", s);
        LAUNCH_R(k_cg_spmv<float>, d.N, s, d, v);
        prof_end("pcg32_spmv", s);
        prof_begin("pcg32_update", s);
        LAUNCH_R(k_cg_update<float>, d.N, s, d, v, 0);
        prof_end("pcg32_update", s);
    } else {
        const BiView<float> v = bi32(d);
        LAUNCH_N(k_bicg_dir<float>, d.N, s, d, v);
        prof_begin("bicg32_spmv", s);
        LAUNCH_R(k_bicg_spmv<float>, d.N, s, d, v);
        prof_end("bicg32_spmv", s);
        LAUNCH_R(k_bicg_update<float>, d.N, s, d, v);
    }
}

void launch_mx_correct_resid(const DevCase &d, int kind, hipStream_t s)
{
    LAUNCH_N(k_mx_correct, d.N, s, d, kind);
    LAUNCH_R(k_mx_resid, d.N, s, d, kind);
}

void launch_dic_precond(const DevCase &d, int with_setup, hipStream_t s)
{
    const int g = cdiv(d.N, kBlock);
    if (with_setup) {
        prof_begin("dic_setup", s);
        hipLaunchKernelGGL(k_dic_sweep<0>, dim3(g), dim3(kBlock), 0, s, d);
        prof_end("dic_setup", s);
    }
    prof_begin("dic_fwd", s);
    hipLaunchKernelGGL(k_dic_sweep<1>, dim3(g), dim3(kBlock), 0, s, d);
    prof_end("dic_fwd", s);
    prof_begin("dic_bwd", s);
    hipLaunchKernelGGL(k_dic_sweep<2>, dim3(g), dim3(kBlock), 0, s, d);
    prof_end("dic_bwd", s);
}

void launch_dic_reset(const DevCase &d, hipStream_t s) { LAUNCH_N(k_dic_reset, d.N, s, d); }

void launch_init_partials(const DevCase &d, hipStream_t s)
{
    const long n = (long)kMaxRed * d.red_stride;
    hipLaunchKernelGGL(k_fill_sentinel, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, s, d.partials, n);
}

void launch_pcg_iter(const DevCase &d, int dic, hipStream_t s)
{
    const CGView<double> v = cg64(d, dic);
    prof_begin("pcg_dir", s);
    LAUNCH_N(k_cg_dir<double>, d.N, s, d, v);
    prof_end("pcg_dir", s);
    prof_begin("pcg_spmv", s);
    LAUNCH_R(k_cg_spmv<double>, d.N, s, d, v);
    prof_end("pcg_spmv", s);
    prof_begin("pcg_update", s);
    LAUNCH_R(k_cg_update<double>, d.N, s, d, v, dic);
    prof_end("pcg_update", s);
    if (dic) launch_dic_precond(d, 0, s);
}

void launch_set_ctl(const DevCase &d, int first, int count, double tol, double rel_tol, int max_iter, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_ctl, dim3(1), dim3(64), 0, s, d.ks, first, count, tol, rel_tol, max_iter);
}

void launch_set_patch(const DevCase &d, int patch, double u0, double u1, double u2, double pv, hipStream_t s)
{
    hipLaunchKernelGGL(k_set_patch, dim3(1), dim3(64), 0, s, d, patch, u0, u1, u2, pv);
}
