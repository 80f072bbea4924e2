// Case lifecycle and the PISO / SIMPLE drivers (host orchestration).
//
// One case = one mesh + options + fields, laid out in a caller-provided
// device workspace.  The drivers enqueue kernels on the caller's stream in
// the order the paper's algorithms prescribe (Section 3): PISO = momentum
// predictor followed by pressure correctors with explicit flux and velocity
// corrections; SIMPLE = the same with under-relaxation and one corrector.
//
// Krylov loop control stays on the device: every iteration kernel reads the
// solve's `done` flag and does nothing once it is set.  The host enqueues
// iterations in chunks and after each chunk an asynchronous copy of the
// Krylov scalars into pinned host memory; it inspects the copy of chunk k
// while chunk k+1 runs, so the GPU never waits for the host and the host
// never synchronises per iteration.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "fvm_internal.h"

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
std::string &fvm_err_buf()
{
    static thread_local std::string s;
    return s;
}

fvm_status fvm_fail(fvm_status code, const std::string &msg)
{
    fvm_err_buf() = msg;
    return code;
}

extern "C" const char *fvm_last_error(void) { return fvm_err_buf().c_str(); }

#define HIPCHK(x)                                                                                   \
    do {                                                                                            \
        hipError_t e_ = (x);                                                                        \
        if (e_ != hipSuccess) return fvm_fail(FVM_EDEVICE, std::string(#x) + ": " + hipGetErrorString(e_)); \
    } while (0)

// ---------------------------------------------------------------------------
// kernel-class timing (measurement only)
// ---------------------------------------------------------------------------
namespace {
struct ProfRec {
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    double ms = 0.0;
    int64_t n = 0;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::map<std::string, ProfRec> g_prof;
std::map<std::string, hipEvent_t> g_prof_open;

void prof_resolve(ProfRec &r)
{
    for (auto &e : r.ev) {
        float ms = 0.f;
        if (hipEventSynchronize(e.second) == hipSuccess && hipEventElapsedTime(&ms, e.first, e.second) == hipSuccess)
            r.ms += ms;
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
        r.n += 1;
    }
    r.ev.clear();
}
}  // namespace

void prof_begin(const char *cls, hipStream_t s)
{
    if (!g_prof_on) return;
    std::lock_guard<std::mutex> g(g_prof_mu);
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    (void)hipEventRecord(e, s);
    g_prof_open[cls] = e;
}

void prof_end(const char *cls, hipStream_t s)
{
    if (!g_prof_on) return;
    std::lock_guard<std::mutex> g(g_prof_mu);
    auto it = g_prof_open.find(cls);
    if (it == g_prof_open.end()) return;
    hipEvent_t e;
    if (hipEventCreate(&e) != hipSuccess) return;
    (void)hipEventRecord(e, s);
    ProfRec &r = g_prof[cls];
    r.ev.emplace_back(it->second, e);
    g_prof_open.erase(it);
    if (r.ev.size() >= 4096) prof_resolve(r);
}

extern "C" fvm_status fvm_profile_enable(int32_t on)
{
    std::lock_guard<std::mutex> g(g_prof_mu);
    if (on) {
        for (auto &kv : g_prof) prof_resolve(kv.second);
        g_prof.clear();
    }
    g_prof_on = on != 0;
    return FVM_OK;
}

extern "C" fvm_status fvm_profile_read(const char *cls, double *total_ms, int64_t *launches)
{
    std::lock_guard<std::mutex> g(g_prof_mu);
    auto it = g_prof.find(cls ? cls : "");
    double ms = 0.0;
    int64_t n = 0;
    if (it != g_prof.end()) {
        prof_resolve(it->second);
        ms = it->second.ms;
        n = it->second.n;
    }
    if (total_ms) *total_ms = ms;
    if (launches) *launches = n;
    return FVM_OK;
}

// ---------------------------------------------------------------------------
// workspace planning: the same walk sizes the workspace and assigns pointers
// ---------------------------------------------------------------------------
namespace {

struct Bump {
    char *base;
    size_t off = 0;
    template <class T>
    T *take(size_t n)
    {
        off = (off + 255) / 256 * 256;
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += sizeof(T) * (n ? n : 1);
        return p;
    }
};

void plan(const fvm_mesh &m, const fvm_case_opts &o, Bump &b, DevCase &d)
{
    const size_t N = m.N, F = m.F, Fi = m.Fi, Fb = m.Fb, np = m.npatch;
    const bool no = m.nonorth, dic = o.p_ctl.precond == FVM_PC_DIC, mixed = o.precision == FVM_MIXED;
    std::memset(&d, 0, sizeof(d));
    d.N = m.N; d.F = m.F; d.Fi = m.Fi; d.Fb = m.Fb; d.npatch = m.npatch;
    d.nonorth = no; d.has_fixed_p = m.has_fixed_p; d.pin_cell = o.p_ref_cell;
    d.n_levels = (int32_t)m.lvl_start.size() - 1;
    d.own = b.take<int32_t>(F); d.nei = b.take<int32_t>(Fi);
    d.own_start = b.take<int32_t>(N + 1); d.nbr_start = b.take<int32_t>(N + 1); d.losort = b.take<int32_t>(Fi);
    d.bnd_start = b.take<int32_t>(N + 1); d.bnd_list = b.take<int32_t>(Fb); d.bpatch = b.take<int32_t>(Fb);
    d.face_user = b.take<int32_t>(Fi); d.face_sign = b.take<int32_t>(Fi);
    d.patch_uk = b.take<int32_t>(np); d.patch_pk = b.take<int32_t>(np);
    d.patch_uv = b.take<double>(3 * np); d.patch_pv = b.take<double>(np);
    d.Sx = b.take<double>(F); d.Sy = b.take<double>(F); d.Sz = b.take<double>(F); d.V = b.take<double>(N);
    d.w = b.take<double>(Fi); d.dl = b.take<double>(F);
    if (no) { d.kx = b.take<double>(Fi); d.ky = b.take<double>(Fi); d.kz = b.take<double>(Fi); }
    d.U = b.take<double>(3 * N); d.p = b.take<double>(N); d.phi = b.take<double>(F); d.p_prev = b.take<double>(N);
    d.U_save = b.take<double>(3 * N); d.p_save = b.take<double>(N); d.phi_save = b.take<double>(F);
    d.mdiag = b.take<double>(N); d.upper = b.take<double>(Fi); d.lower = b.take<double>(Fi);
    d.src = b.take<double>(3 * N); d.rhs = b.take<double>(3 * N);
    if (no) { d.gradU = b.take<double>(9 * N); d.ns = b.take<double>(3 * Fi); d.tno = b.take<double>(Fi); }
    d.rAU = b.take<double>(N); d.HbyA = b.take<double>(3 * N); d.gradp = b.take<double>(3 * N);
    d.phiH = b.take<double>(F); d.gam = b.take<double>(F); d.pdiag = b.take<double>(N); d.poff = b.take<double>(Fi);
    d.pb = b.take<double>(N);
    // Krylov vectors; the setup temporaries (cell and face centres) alias them
    const size_t kv = std::max(18 * N, 3 * N + 3 * F);
    double *kbase = b.take<double>(kv);
    if (kbase) {
        d.r = kbase; d.rt = kbase + 3 * N; d.pp = kbase + 6 * N; d.pt = kbase + 9 * N; d.q = kbase + 12 * N;
        d.qt = kbase + 15 * N;
        d.tmpC = kbase; d.tmpCf = kbase + 3 * N;
    }
    if (dic) {
        d.y = b.take<double>(N); d.z = b.take<double>(N); d.dstar = b.take<double>(N);
        d.lvl_start = b.take<int32_t>(m.lvl_start.size()); d.lvl_cells = b.take<int32_t>(N);
    }
    if (mixed) {
        d.f_diag = b.take<float>(N); d.f_up = b.take<float>(Fi); d.f_lo = b.take<float>(Fi);
        d.f_pdiag = b.take<float>(N); d.f_poff = b.take<float>(Fi);
        d.f_x = b.take<float>(3 * N); d.f_b = b.take<float>(3 * N); d.f_r = b.take<float>(3 * N);
        d.f_rt = b.take<float>(3 * N); d.f_p = b.take<float>(3 * N); d.f_pt = b.take<float>(3 * N);
        d.f_q = b.take<float>(3 * N); d.f_qt = b.take<float>(3 * N);
    }
    d.red_stride = std::max<int32_t>(kMaxGrid, (int32_t)((N + kBlock - 1) / kBlock));
    d.partials = b.take<double>((size_t)kMaxRed * d.red_stride);
    d.ticket = b.take<unsigned int>(64);
    d.ks = b.take<KState>(kNumKs);
    b.off = (b.off + 255) / 256 * 256;
}

fvm_status check_opts(const fvm_mesh *m, const fvm_case_opts *o)
{
    if (!m || !o) return fvm_fail(FVM_EINVAL, "case: null mesh or options");
    if (!(o->nu > 0.0) || !std::isfinite(o->nu)) return fvm_fail(FVM_EINVAL, "case: nu must be > 0");
    if (o->n_corr < 1 || o->n_non_orth_corr < 0 || o->n_corr * (o->n_non_orth_corr + 1) > 16)
        return fvm_fail(FVM_EINVAL, "case: need 1 <= n_corr*(n_non_orth_corr+1) <= 16");
    if (o->p_ref_cell < 0 || o->p_ref_cell >= m->N) return fvm_fail(FVM_EINVAL, "case: p_ref_cell out of range");
    if (o->precision != FVM_FP64 && o->precision != FVM_MIXED) return fvm_fail(FVM_EINVAL, "case: bad precision");
    if (o->precision == FVM_MIXED && o->p_ctl.precond == FVM_PC_DIC)
        return fvm_fail(FVM_EINVAL, "case: mixed precision runs Jacobi inner solves (DIC is FP64 only)");
    if (o->precision == FVM_MIXED && (!(o->inner_rel_tol > 0.0) || !(o->inner_rel_tol < 1.0) || o->inner_max_iter < 1))
        return fvm_fail(FVM_EINVAL, "case: mixed precision needs 0 < inner_rel_tol < 1 and inner_max_iter >= 1");
    if (o->p_ctl.precond != FVM_PC_JACOBI && o->p_ctl.precond != FVM_PC_DIC)
        return fvm_fail(FVM_EINVAL, "case: bad preconditioner");
    if (o->u_ctl.precond != FVM_PC_JACOBI) return fvm_fail(FVM_EINVAL, "case: momentum solver takes Jacobi only");
    if (o->p_ctl.max_iter < 1 || o->u_ctl.max_iter < 1) return fvm_fail(FVM_EINVAL, "case: max_iter must be >= 1");
    if (!(o->p_ctl.tol >= 0.0) || !(o->u_ctl.tol >= 0.0) || !(o->p_ctl.rel_tol >= 0.0) || !(o->u_ctl.rel_tol >= 0.0))
        return fvm_fail(FVM_EINVAL, "case: tolerances must be >= 0");
    if (o->convection != FVM_CONV_LINEAR && o->convection != FVM_CONV_UPWIND)
        return fvm_fail(FVM_EINVAL, "case: bad convection scheme");
    return FVM_OK;
}

constexpr int kRing = 4;

}  // namespace

struct fvm_case {
    fvm_case_opts o;
    DevCase d;
    int32_t N, F, Fi, Fb, npatch;
    bool nonorth, has_fixed_p;
    std::vector<fvm_patch> patches;
    // Krylov state mirror: a ring of pinned host copies, one per chunk
    KState *hks = nullptr;          // [kRing][kNumKs]
    hipEvent_t ev[kRing];
    bool ev_pending[kRing];
    int ring = 0;
    int last_iters[4] = {0, 0, 0, 0};   // momentum, pressure, and their inner solves: chunk sizing
};

// ---------------------------------------------------------------------------
// public: workspace size, create, destroy
// ---------------------------------------------------------------------------
extern "C" fvm_status fvm_case_workspace_bytes(const fvm_mesh *m, const fvm_case_opts *o, size_t *bytes)
{
    fvm_status st = check_opts(m, o);
    if (st != FVM_OK) return st;
    if (!bytes) return fvm_fail(FVM_EINVAL, "case: null output");
    Bump b{nullptr};
    DevCase d;
    plan(*m, *o, b, d);
    *bytes = b.off;
    return FVM_OK;
}

namespace {
template <class T>
hipError_t up(T *dst, const std::vector<T> &src, hipStream_t s)
{
    if (src.empty()) return hipSuccess;
    return hipMemcpyAsync(dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice, s);
}

fvm_status upload_patches(fvm_case *c, hipStream_t s)
{
    const int np = c->npatch;
    if (np == 0) return FVM_OK;
    std::vector<int32_t> uk(np), pk(np);
    std::vector<double> uv(3 * (size_t)np), pv(np);
    for (int p = 0; p < np; ++p) {
        uk[p] = c->patches[p].u_kind; pk[p] = c->patches[p].p_kind; pv[p] = c->patches[p].p_value;
        for (int k = 0; k < 3; ++k) uv[3 * p + k] = c->patches[p].u_value[k];
    }
    HIPCHK(up(c->d.patch_uk, uk, s));
    HIPCHK(up(c->d.patch_pk, pk, s));
    HIPCHK(up(c->d.patch_uv, uv, s));
    HIPCHK(up(c->d.patch_pv, pv, s));
    HIPCHK(hipStreamSynchronize(s));    // the host vectors above are temporaries
    return FVM_OK;
}
}  // namespace

extern "C" fvm_status fvm_case_create(const fvm_mesh *m, const fvm_case_opts *o, void *ws, size_t bytes, void *stream,
                                      fvm_case **out)
{
    if (!out) return fvm_fail(FVM_EINVAL, "case: null output");
    *out = nullptr;
    fvm_status st = check_opts(m, o);
    if (st != FVM_OK) return st;
    if (!ws || (reinterpret_cast<uintptr_t>(ws) & 255)) return fvm_fail(FVM_EINVAL, "case: workspace must be 256-byte aligned");
    size_t need = 0;
    fvm_case_workspace_bytes(m, o, &need);
    if (bytes < need) return fvm_fail(FVM_ENOMEM, "case: workspace too small (" + std::to_string(bytes) + " < " + std::to_string(need) + ")");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    fvm_case *c = new (std::nothrow) fvm_case();
    if (!c) return fvm_fail(FVM_ENOMEM, "case: out of host memory");
    c->o = *o;
    c->N = m->N; c->F = m->F; c->Fi = m->Fi; c->Fb = m->Fb; c->npatch = m->npatch;
    c->nonorth = m->nonorth; c->has_fixed_p = m->has_fixed_p;
    c->patches = m->patches;
    Bump b{reinterpret_cast<char *>(ws)};
    plan(*m, *o, b, c->d);
    auto fail = [&](fvm_status code) {
        if (c->hks) (void)hipHostFree(c->hks);
        delete c;
        return code;
    };
    if (hipHostMalloc((void **)&c->hks, sizeof(KState) * kNumKs * kRing, hipHostMallocDefault) != hipSuccess)
        return fail(fvm_fail(FVM_EDEVICE, "case: pinned host buffer"));
    for (int k = 0; k < kRing; ++k) {
        c->ev_pending[k] = false;
        if (hipEventCreateWithFlags(&c->ev[k], hipEventDisableTiming) != hipSuccess)
            return fail(fvm_fail(FVM_EDEVICE, "case: event"));
    }
    DevCase &d = c->d;
    const size_t N = m->N, F = m->F;
#define UPCHK(x) do { if ((x) != hipSuccess) return fail(fvm_fail(FVM_EDEVICE, "case: upload " #x)); } while (0)
    UPCHK(up(d.own, m->own, s)); UPCHK(up(d.nei, m->nei, s));
    UPCHK(up(d.own_start, m->own_start, s)); UPCHK(up(d.nbr_start, m->nbr_start, s)); UPCHK(up(d.losort, m->losort, s));
    UPCHK(up(d.bnd_start, m->bnd_start, s)); UPCHK(up(d.bnd_list, m->bnd_list, s)); UPCHK(up(d.bpatch, m->bpatch, s));
    UPCHK(up(d.face_user, m->face_user, s)); UPCHK(up(d.face_sign, m->face_sign, s));
    UPCHK(hipMemcpyAsync(d.Sx, m->S.data(), sizeof(double) * F, hipMemcpyHostToDevice, s));
    UPCHK(hipMemcpyAsync(d.Sy, m->S.data() + F, sizeof(double) * F, hipMemcpyHostToDevice, s));
    UPCHK(hipMemcpyAsync(d.Sz, m->S.data() + 2 * F, sizeof(double) * F, hipMemcpyHostToDevice, s));
    UPCHK(up(d.V, m->V, s));
    UPCHK(up(d.tmpC, m->C, s));
    UPCHK(up(d.tmpCf, m->Cf, s));
    if (d.lvl_start) { UPCHK(up(d.lvl_start, m->lvl_start, s)); UPCHK(up(d.lvl_cells, m->lvl_cells, s)); }
    UPCHK(hipMemsetAsync(d.ticket, 0, 64 * sizeof(unsigned int), s));
    UPCHK(hipMemsetAsync(d.ks, 0, kNumKs * sizeof(KState), s));
    st = upload_patches(c, s);
    if (st != FVM_OK) return fail(st);
    launch_init_partials(d, s);
    launch_geometry(d, s);
    UPCHK(hipMemsetAsync(d.U, 0, 3 * N * sizeof(double), s));
    UPCHK(hipMemsetAsync(d.p, 0, N * sizeof(double), s));
    launch_flux_from_U(d, s);
    UPCHK(hipGetLastError());
    UPCHK(hipStreamSynchronize(s));   // the mesh vectors may be freed by the caller after return
#undef UPCHK
    *out = c;
    return FVM_OK;
}

extern "C" void fvm_case_destroy(fvm_case *c)
{
    if (!c) return;
    for (int k = 0; k < kRing; ++k) (void)hipEventDestroy(c->ev[k]);
    if (c->hks) (void)hipHostFree(c->hks);
    delete c;
}

// ---------------------------------------------------------------------------
// public: state exchange
// ---------------------------------------------------------------------------
extern "C" fvm_status fvm_case_set_state(fvm_case *c, const double *U, const double *p, const double *phi, void *stream)
{
    if (!c) return fvm_fail(FVM_EINVAL, "case: null handle");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (U) launch_U_in(c->d, U, s);
    if (p) HIPCHK(hipMemcpyAsync(c->d.p, p, sizeof(double) * c->N, hipMemcpyDeviceToDevice, s));
    if (phi) launch_phi_in(c->d, phi, s);
    else launch_flux_from_U(c->d, s);
    HIPCHK(hipGetLastError());
    return FVM_OK;
}

extern "C" fvm_status fvm_case_get_state(const fvm_case *c, double *U, double *p, double *phi, void *stream)
{
    if (!c) return fvm_fail(FVM_EINVAL, "case: null handle");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (U) launch_U_out(c->d, U, s);
    if (p) HIPCHK(hipMemcpyAsync(p, c->d.p, sizeof(double) * c->N, hipMemcpyDeviceToDevice, s));
    if (phi) launch_phi_out(c->d, phi, s);
    HIPCHK(hipGetLastError());
    return FVM_OK;
}

extern "C" fvm_status fvm_case_set_patch_value(fvm_case *c, int32_t patch, const double u_value[3], double p_value,
                                               void *stream)
{
    if (!c) return fvm_fail(FVM_EINVAL, "case: null handle");
    if (patch < 0 || patch >= c->npatch || !u_value) return fvm_fail(FVM_EINVAL, "case: bad patch index");
    for (int k = 0; k < 3; ++k) c->patches[patch].u_value[k] = u_value[k];
    c->patches[patch].p_value = p_value;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    launch_set_patch(c->d, patch, u_value[0], u_value[1], u_value[2], p_value, s);
    HIPCHK(hipGetLastError());
    return FVM_OK;
}

// ---------------------------------------------------------------------------
// Krylov drivers
// ---------------------------------------------------------------------------
namespace {

struct SolveOut {
    KState ks[4];
};

// Enqueue iterations in chunks until the systems [first, first+count) are
// done; the Krylov state array after the last chunk is returned in res.
// launch_iter enqueues one iteration.  `predicted` sizes the first chunk.
template <class F>
fvm_status iterate_until_done(fvm_case *c, int first, int count, int predicted, long limit, hipStream_t s,
                              F launch_iter, KState *res)
{
    const DevCase &d = c->d;
    int chunk = predicted > 0 ? std::max(2, predicted - predicted / 4) : 4;
    long issued = 0;
    int prev_slot = -1;
    auto all_done = [&](const KState *h) {
        for (int k = 0; k < count; ++k)
            if (!h[first + k].done) return false;
        return true;
    };
    for (;;) {
        const int n = (int)std::min<long>(chunk, std::max<long>(1, limit - issued));
        for (int k = 0; k < n; ++k) launch_iter();
        issued += n;
        HIPCHK(hipGetLastError());
        const int slot = c->ring;
        c->ring = (c->ring + 1) % kRing;
        if (c->ev_pending[slot]) {
            HIPCHK(hipEventSynchronize(c->ev[slot]));
            c->ev_pending[slot] = false;
        }
        HIPCHK(hipMemcpyAsync(c->hks + kNumKs * slot, d.ks, kNumKs * sizeof(KState), hipMemcpyDeviceToHost, s));
        HIPCHK(hipEventRecord(c->ev[slot], s));
        c->ev_pending[slot] = true;
        // inspect the previous chunk while this one runs
        if (prev_slot >= 0) {
            HIPCHK(hipEventSynchronize(c->ev[prev_slot]));
            c->ev_pending[prev_slot] = false;
            if (all_done(c->hks + kNumKs * prev_slot)) {
                std::memcpy(res, c->hks + kNumKs * prev_slot, kNumKs * sizeof(KState));
                return FVM_OK;
            }
        }
        if (issued >= limit) {
            HIPCHK(hipEventSynchronize(c->ev[slot]));
            c->ev_pending[slot] = false;
            std::memcpy(res, c->hks + kNumKs * slot, kNumKs * sizeof(KState));
            if (!all_done(res)) return fvm_fail(FVM_EDEVICE, "solve: iteration limit passed without a stop flag");
            return FVM_OK;
        }
        prev_slot = slot;
        chunk = predicted > 0 ? std::max(2, predicted / 8) : std::min(64, chunk * 2);
    }
}

// synchronous copy of the Krylov states (once per outer refinement step)
fvm_status snapshot(fvm_case *c, hipStream_t s, KState *res)
{
    const int slot = c->ring;
    c->ring = (c->ring + 1) % kRing;
    if (c->ev_pending[slot]) {
        HIPCHK(hipEventSynchronize(c->ev[slot]));
        c->ev_pending[slot] = false;
    }
    HIPCHK(hipMemcpyAsync(c->hks + kNumKs * slot, c->d.ks, kNumKs * sizeof(KState), hipMemcpyDeviceToHost, s));
    HIPCHK(hipEventRecord(c->ev[slot], s));
    HIPCHK(hipEventSynchronize(c->ev[slot]));
    std::memcpy(res, c->hks + kNumKs * slot, kNumKs * sizeof(KState));
    return FVM_OK;
}

// Enqueue one solve and return its final scalars.  kind 0: momentum BiCG
// (systems 0..2), kind 1: pressure CG (system 3).  FVM_MIXED cases run the
// FP64 refinement loop around FP32 inner solves (systems 4..7).
fvm_status run_solve(fvm_case *c, int kind, const fvm_solver_ctl &ctl, hipStream_t s, KState *final_state)
{
    const DevCase &d = c->d;
    const int first = kind == 0 ? 0 : 3, count = kind == 0 ? 3 : 1;
    const int dic = kind == 1 && ctl.precond == FVM_PC_DIC;
    const bool mixed = c->o.precision == FVM_MIXED;
    launch_set_ctl(d, first, count, ctl.tol, ctl.rel_tol, ctl.max_iter, s);
    if (kind == 0) launch_bicg_init(d, s);
    else launch_pcg_init(d, dic, s);
    KState res[kNumKs];
    fvm_status st;
    if (!mixed) {
        if (dic) launch_dic_precond(d, 1, s);
        st = iterate_until_done(c, first, count, c->last_iters[kind], (long)ctl.max_iter + 1, s, [&] {
            if (kind == 0) launch_bicg_iter(d, s);
            else launch_pcg_iter(d, dic, s);
        }, res);
        if (st != FVM_OK) return st;
    } else {
        const int ifirst = kind == 0 ? 4 : 7;
        launch_set_ctl(d, ifirst, count, 0.0, c->o.inner_rel_tol, c->o.inner_max_iter, s);
        launch_mx_cvt(d, kind, s);
        for (int outer = 0;; ++outer) {
            st = snapshot(c, s, res);
            if (st != FVM_OK) return st;
            bool all = true;
            for (int k = 0; k < count; ++k) all = all && res[first + k].done;
            if (all) break;
            if (outer >= 1000) return fvm_fail(FVM_EDEVICE, "solve: refinement did not terminate");
            launch_mx_inner_init(d, kind, s);
            st = iterate_until_done(c, ifirst, count, c->last_iters[2 + kind], (long)c->o.inner_max_iter + 1, s,
                                    [&] { launch_mx_inner_iter(d, kind, s); }, res);
            if (st != FVM_OK) return st;
            int mi = 0;
            for (int k = 0; k < count; ++k) mi = std::max(mi, res[ifirst + k].iters);
            c->last_iters[2 + kind] = mi;
            launch_mx_correct_resid(d, kind, s);
        }
    }
    int mx = 0;
    for (int k = 0; k < count; ++k) mx = std::max(mx, res[first + k].iters);
    c->last_iters[kind] = mx;
    for (int k = 0; k < count; ++k) final_state[k] = res[first + k];
    return FVM_OK;
}

void to_info(const KState &k, fvm_solve_info &i)
{
    i.iters = k.iters;
    i.status = k.status;
    i.res_initial = k.nres0;
    i.res_final = k.nres;
}

void worst(int32_t &acc, int32_t s)
{
    if (s < 0) { if (acc >= 0 || s < acc) acc = s; }
    else if (acc >= 0 && s > acc) acc = s;
}

fvm_status save_state(fvm_case *c, hipStream_t s)
{
    const DevCase &d = c->d;
    HIPCHK(hipMemcpyAsync(d.U_save, d.U, 3 * sizeof(double) * c->N, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(d.p_save, d.p, sizeof(double) * c->N, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(d.phi_save, d.phi, sizeof(double) * c->F, hipMemcpyDeviceToDevice, s));
    return FVM_OK;
}

fvm_status restore_state(fvm_case *c, hipStream_t s)
{
    const DevCase &d = c->d;
    HIPCHK(hipMemcpyAsync(d.U, d.U_save, 3 * sizeof(double) * c->N, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(d.p, d.p_save, sizeof(double) * c->N, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(d.phi, d.phi_save, sizeof(double) * c->F, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return FVM_OK;
}

// momentum matrix + predictor solve; dt > 0 transient, alpha_u < 1 relaxed
fvm_status momentum_predictor(fvm_case *c, double dt, double alpha_u, hipStream_t s, fvm_step_info &info)
{
    const DevCase &d = c->d;
    const int upwind = c->o.convection == FVM_CONV_UPWIND;
    if (c->nonorth) launch_gradU(d, s);
    launch_mom_face(d, c->o.nu, upwind, s);
    launch_mom_cell(d, c->o.nu, dt, alpha_u, upwind, s);
    KState ks[3];
    fvm_status st = run_solve(c, 0, c->o.u_ctl, s, ks);
    if (st != FVM_OK) return st;
    for (int k = 0; k < 3; ++k) {
        to_info(ks[k], info.u[k]);
        worst(info.status, ks[k].status);
    }
    return FVM_OK;
}

// one pressure solve on the assembled system, recorded in info
fvm_status pressure_solve(fvm_case *c, const fvm_solver_ctl &ctl, hipStream_t s, fvm_step_info &info)
{
    KState ks;
    fvm_status st = run_solve(c, 1, ctl, s, &ks);
    if (st != FVM_OK) return st;
    if (info.n_p_solves < 16) to_info(ks, info.p[info.n_p_solves++]);
    worst(info.status, ks.status);
    return FVM_OK;
}

fvm_status piso_one(fvm_case *c, hipStream_t s, fvm_step_info &info)
{
    const DevCase &d = c->d;
    std::memset(&info, 0, sizeof(info));
    fvm_status st = momentum_predictor(c, c->o.dt, 1.0, s, info);
    if (st != FVM_OK || info.status < 0) return st;
    for (int corr = 0; corr < c->o.n_corr; ++corr) {
        for (int k = 0; k <= c->o.n_non_orth_corr; ++k) {
            if (k == 0) launch_hbya(d, c->nonorth, s);
            else launch_gradp(d, s);
            launch_p_face(d, s);
            launch_p_cell(d, c->o.p_ref_value, s);
            st = pressure_solve(c, c->o.p_ctl, s, info);
            if (st != FVM_OK || info.status < 0) return st;
        }
        launch_flux_corr(d, s);
        launch_U_corr(d, s);
    }
    HIPCHK(hipGetLastError());
    return FVM_OK;
}

fvm_status simple_one(fvm_case *c, hipStream_t s, fvm_step_info &info)
{
    const DevCase &d = c->d;
    std::memset(&info, 0, sizeof(info));
    fvm_status st = momentum_predictor(c, 0.0, c->o.alpha_u, s, info);
    if (st != FVM_OK || info.status < 0) return st;
    HIPCHK(hipMemcpyAsync(d.p_prev, d.p, sizeof(double) * c->N, hipMemcpyDeviceToDevice, s));
    launch_hbya(d, c->nonorth, s);
    launch_p_face(d, s);
    launch_p_cell(d, c->o.p_ref_value, s);
    st = pressure_solve(c, c->o.p_ctl, s, info);
    if (st != FVM_OK || info.status < 0) return st;
    launch_flux_corr(d, s);
    launch_p_relax(d, c->o.alpha_p, s);
    launch_U_corr(d, s);
    HIPCHK(hipGetLastError());
    return FVM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// public: PISO, SIMPLE, stand-alone pressure solve, batch
// ---------------------------------------------------------------------------
extern "C" fvm_status piso_step(fvm_case *c, int32_t n_steps, void *stream, fvm_step_info *last)
{
    if (!c) return fvm_fail(FVM_EINVAL, "piso: null handle");
    if (n_steps < 0) return fvm_fail(FVM_EINVAL, "piso: n_steps < 0");
    if (!(c->o.dt > 0.0)) return fvm_fail(FVM_EINVAL, "piso: dt must be > 0");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int32_t acc = FVM_OK;
    fvm_step_info info;
    std::memset(&info, 0, sizeof(info));
    for (int32_t k = 0; k < n_steps; ++k) {
        fvm_status st = save_state(c, s);
        if (st != FVM_OK) return st;
        st = piso_one(c, s, info);
        if (st == FVM_OK && info.status < 0) st = fvm_fail(info.status, "piso: a solve failed (non-finite value or breakdown)");
        if (st < 0) {
            restore_state(c, s);
            if (last) *last = info;
            return st;
        }
        worst(acc, info.status);
    }
    if (last) *last = info;
    return acc;
}

extern "C" fvm_status simple_iterate(fvm_case *c, int32_t max_iters, double res_tol, void *stream, int32_t *iters_done,
                                     fvm_step_info *last)
{
    if (!c) return fvm_fail(FVM_EINVAL, "simple: null handle");
    if (max_iters < 0) return fvm_fail(FVM_EINVAL, "simple: max_iters < 0");
    if (!(c->o.alpha_u > 0.0 && c->o.alpha_u <= 1.0) || !(c->o.alpha_p > 0.0 && c->o.alpha_p <= 1.0))
        return fvm_fail(FVM_EINVAL, "simple: relaxation factors must be in (0, 1]");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    int32_t acc = FVM_OK, it = 0;
    fvm_step_info info;
    std::memset(&info, 0, sizeof(info));
    for (it = 0; it < max_iters;) {
        fvm_status st = save_state(c, s);
        if (st != FVM_OK) return st;
        st = simple_one(c, s, info);
        if (st == FVM_OK && info.status < 0) st = fvm_fail(info.status, "simple: a solve failed (non-finite value or breakdown)");
        if (st < 0) {
            restore_state(c, s);
            if (iters_done) *iters_done = it;
            if (last) *last = info;
            return st;
        }
        ++it;
        worst(acc, info.status);
        if (info.u[0].res_initial <= res_tol && info.u[1].res_initial <= res_tol && info.u[2].res_initial <= res_tol &&
            info.p[0].res_initial <= res_tol)
            break;
    }
    if (iters_done) *iters_done = it;
    if (last) *last = info;
    return acc;
}

extern "C" fvm_status solve_pressure(fvm_case *c, const double *gamma, const double *rhs, double *p,
                                     const fvm_solver_ctl *ctl, void *stream, fvm_solve_info *out)
{
    if (!c || !gamma || !rhs || !p || !ctl) return fvm_fail(FVM_EINVAL, "solve_pressure: null argument");
    if (ctl->precond != FVM_PC_JACOBI && ctl->precond != FVM_PC_DIC)
        return fvm_fail(FVM_EINVAL, "solve_pressure: bad preconditioner");
    if (ctl->precond == FVM_PC_DIC && !c->d.dstar)
        return fvm_fail(FVM_EINVAL, "solve_pressure: DIC needs a case created with the DIC preconditioner");
    if (ctl->max_iter < 1) return fvm_fail(FVM_EINVAL, "solve_pressure: max_iter must be >= 1");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const DevCase &d = c->d;
    // the case's p field is the solver's unknown: park it
    HIPCHK(hipMemcpyAsync(d.p_save, d.p, sizeof(double) * c->N, hipMemcpyDeviceToDevice, s));
    launch_gather_faces(d, gamma, d.phiH, s);
    launch_p_system_from_gamma(d, d.phiH, rhs, c->o.p_ref_value, s);
    HIPCHK(hipMemcpyAsync(d.p, p, sizeof(double) * c->N, hipMemcpyDeviceToDevice, s));
    KState ks;
    fvm_status st = run_solve(c, 1, *ctl, s, &ks);
    if (st != FVM_OK) return st;
    if (ks.status >= 0) HIPCHK(hipMemcpyAsync(p, d.p, sizeof(double) * c->N, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(d.p, d.p_save, sizeof(double) * c->N, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    if (out) to_info(ks, *out);
    if (ks.status < 0) return fvm_fail(ks.status, "solve_pressure: non-finite value or breakdown");
    return ks.status;
}

extern "C" fvm_status fvm_dic_apply(fvm_case *c, const double *gamma, const double *r, double *z, double *dstar,
                                    void *stream)
{
    if (!c || !gamma || !r || !z) return fvm_fail(FVM_EINVAL, "dic_apply: null argument");
    if (!c->d.dstar) return fvm_fail(FVM_EINVAL, "dic_apply: case was not created with the DIC preconditioner");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const DevCase &d = c->d;
    launch_gather_faces(d, gamma, d.phiH, s);
    launch_p_system_from_gamma(d, d.phiH, r, c->o.p_ref_value, s);
    HIPCHK(hipMemcpyAsync(d.r, r, sizeof(double) * c->N, hipMemcpyDeviceToDevice, s));
    launch_dic_reset(d, s);
    launch_dic_precond(d, 1, s);
    HIPCHK(hipMemcpyAsync(z, d.z, sizeof(double) * c->N, hipMemcpyDeviceToDevice, s));
    if (dstar) HIPCHK(hipMemcpyAsync(dstar, d.dstar, sizeof(double) * c->N, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return FVM_OK;
}

extern "C" fvm_status piso_step_batch(fvm_case *const *cases, int32_t n, int32_t n_steps, void *stream,
                                      fvm_step_info *infos)
{
    if (!cases || n < 0) return fvm_fail(FVM_EINVAL, "batch: bad arguments");
    int32_t acc = FVM_OK;
    for (int32_t i = 0; i < n; ++i) {
        fvm_status st = piso_step(cases[i], n_steps, stream, infos ? infos + i : nullptr);
        if (st < 0) return st;
        worst(acc, st);
    }
    return acc;
}
