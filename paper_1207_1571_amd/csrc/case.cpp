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
#include <rocprofiler-sdk-roctx/roctx.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
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

void plan(const fvm_mesh &m, const fvm_case_opts &o, Bump &b, DevCase &d, std::vector<AmgLevel> *lv = nullptr)
{
    const size_t N = m.N, F = m.F, Fi = m.Fi, Fb = m.Fb, np = m.npatch;
    const bool no = m.nonorth, dic = o.p_ctl.precond == FVM_PC_DIC, mixed = o.precision == FVM_MIXED;
    std::memset(&d, 0, sizeof(d));
    d.N = m.N; d.F = m.F; d.Fi = m.Fi; d.Fb = m.Fb; d.npatch = m.npatch;
    d.nonorth = no; d.has_fixed_p = m.has_fixed_p; d.pin_cell = o.p_ref_cell;
    d.nu = o.nu; d.dt = o.dt; d.alpha_u = o.alpha_u; d.alpha_p = o.alpha_p; d.p_ref = o.p_ref_value;
    d.inner_rel_tol = o.inner_rel_tol; d.inner_max_iter = o.inner_max_iter;
    d.upwind = o.convection == FVM_CONV_UPWIND;
    d.u_tol = o.u_ctl.tol; d.u_rel_tol = o.u_ctl.rel_tol; d.u_max_iter = o.u_ctl.max_iter;
    d.p_tol = o.p_ctl.tol; d.p_rel_tol = o.p_ctl.rel_tol; d.p_max_iter = o.p_ctl.max_iter;
    d.n_levels = (int32_t)m.lvl_start.size() - 1;
    {
        // a wave of the DIC sweeps starts polling once the position this far
        // before its first one is done: two of the widest levels, at least
        // 8192 positions (128 waves), in whole waves
        int32_t wmax = 0;
        for (int32_t l = 0; l < d.n_levels; ++l) wmax = std::max(wmax, m.lvl_start[l + 1] - m.lvl_start[l]);
        d.dic_lag = ((std::max<int32_t>(8192, 2 * wmax) + 63) / 64) * 64;
    }
    d.self = b.take<DevCase>(1);
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
    // Krylov vectors; the setup temporaries (cell and face centres) alias them.
    // BiCGStab: r, r~, p, v, s, t in r..qt, and p^, s^ after them
    const bool stab = o.u_solver == FVM_SOLVER_BICGSTAB;
    d.u_stab = stab;
    const size_t kv = std::max((stab ? 24 : 18) * N, 3 * N + 3 * F);
    double *kbase = b.take<double>(kv);
    if (kbase) {
        d.r = kbase; d.rt = kbase + 3 * N; d.pp = kbase + 6 * N; d.pt = kbase + 9 * N; d.q = kbase + 12 * N;
        d.qt = kbase + 15 * N;
        if (stab) { d.ph = kbase + 18 * N; d.sh = kbase + 21 * N; }
        d.tmpC = kbase; d.tmpCf = kbase + 3 * N;
    }
    if (dic) {
        d.z = b.take<double>(N); d.dstar = b.take<double>(N);
        d.dq = b.take<double>(N); d.yq = b.take<double>(N); d.zq = b.take<double>(N);
        d.lvl_cells = b.take<int32_t>(N);
        d.dW_lo = m.dW_lo; d.dW_hi = m.dW_hi;
        d.dl_pos = b.take<int32_t>((size_t)m.dW_lo * N); d.dl_face = b.take<int32_t>((size_t)m.dW_lo * N);
        d.du_pos = b.take<int32_t>((size_t)m.dW_hi * N); d.du_face = b.take<int32_t>((size_t)m.dW_hi * N);
        d.dl_val = b.take<double>((size_t)m.dW_lo * N); d.du_val = b.take<double>((size_t)m.dW_hi * N);
    }
    if (mixed) {
        d.f_diag = b.take<float>(N); d.f_up = b.take<float>(Fi); d.f_lo = b.take<float>(Fi);
        d.f_pdiag = b.take<float>(N); d.f_poff = b.take<float>(Fi); d.f_pexc = b.take<float>(N);
        d.f_x = b.take<float>(3 * N); d.f_r = b.take<float>(3 * N);
        d.f_rt = b.take<float>(3 * N); d.f_p = b.take<float>(3 * N); d.f_pt = b.take<float>(3 * N);
        d.f_q = b.take<float>(3 * N); d.f_qt = b.take<float>(3 * N);
    }
    {
        const size_t ns = (N + kBlock - 1) / kBlock, W = (size_t)m.sell_W;
        d.sell_W = m.sell_W;
        d.sell_n7 = m.sell_n7;
        d.sell_mode = b.take<int32_t>(ns); d.sell_off = b.take<int32_t>(ns * W); d.sell_mir = b.take<int32_t>(ns * W);
        d.sell_fe = b.take<int32_t>(ns * W * kBlock); d.sell_col = b.take<int32_t>(ns * W * kBlock);
        if (mixed) d.f_sell_val = b.take<float>(ns * W * kBlock);
        else d.sell_val = b.take<double>(ns * W * kBlock);
    }
    if (o.p_ctl.precond == FVM_PC_AMG) {
        const AmgHost &A = mesh_amg(m);
        const int nl = (int)A.L.size();
        d.amg_nl = nl;
        d.amg_nc = A.L[nl - 1].n;
        d.amg = b.take<AmgLevel>(nl);
        d.amg_cinv = b.take<double>((size_t)d.amg_nc * d.amg_nc);
        d.amg_img = b.take<double>(kAmgTailLds / 8);
        if (!d.z) d.z = b.take<double>(N);
        std::vector<AmgLevel> tmp;
        std::vector<AmgLevel> &v = lv ? *lv : tmp;
        v.assign(nl, AmgLevel{});
        for (int l = 0; l < nl; ++l) {
            const AmgLevelHost &L = A.L[l];
            const size_t n = L.n, nf = L.nf;
            d.amg_n[l] = L.n;
            d.amg_nf[l] = L.nf;
            AmgLevel &e = v[l];
            e.n = L.n;
            e.nf = L.nf;
            e.x = b.take<double>(n);
            e.r = b.take<double>(n);
            if (l > 0) {
                e.diag = b.take<double>(n); e.offd = b.take<double>(nf); e.b = b.take<double>(n);
                e.out = e.r;
                e.own = b.take<int32_t>(nf); e.nei = b.take<int32_t>(nf);
                e.own_start = b.take<int32_t>(n + 1); e.nbr_start = b.take<int32_t>(n + 1);
                e.losort = b.take<int32_t>(nf);
                e.mstart = b.take<int32_t>(L.mstart.size()); e.members = b.take<int32_t>(L.members.size());
                e.istart = b.take<int32_t>(L.istart.size()); e.inner = b.take<int32_t>(L.inner.size());
                e.cstart = b.take<int32_t>(L.cstart.size()); e.cfaces = b.take<int32_t>(L.cfaces.size());
            } else {
                e.diag = d.pdiag; e.offd = d.poff; e.b = d.r; e.out = d.z;
                e.own = d.own; e.nei = d.nei; e.own_start = d.own_start; e.nbr_start = d.nbr_start;
                e.losort = d.losort;
            }
            if (l < nl - 1) e.agg = b.take<int32_t>(n);
            d.amg_b[l] = e.b;
            d.amg_out[l] = e.out;
        }
    }
    if (o.hybrid_K > 0) {
        const size_t K = (size_t)o.hybrid_K;
        size_t nC = 0;
        for (int32_t i = 0; i < m.N; ++i) {
            const size_t len = (size_t)(m.nbr_start[i + 1] - m.nbr_start[i]) + 1 + (m.own_start[i + 1] - m.own_start[i]);
            nC += len > K ? len - K : 0;
        }
        const size_t E = K * N + nC;
        d.hy_K = o.hybrid_K; d.hy_nC = (int32_t)nC;
        d.hy_I = b.take<int32_t>(K * N); d.hy_J = b.take<int32_t>(K * N); d.hy_dpos = b.take<int32_t>(N);
        d.hy_locO = b.take<int32_t>(Fi); d.hy_locN = b.take<int32_t>(Fi);
        d.hy_cstart = b.take<int32_t>(N + 1); d.hy_ccol = b.take<int32_t>(nC); d.hy_ctrpos = b.take<int32_t>(nC);
        d.hy_V = b.take<double>(E); d.hy_Sx = b.take<double>(E); d.hy_Sy = b.take<double>(E); d.hy_Sz = b.take<double>(E);
        d.hy_w = b.take<double>(E); d.hy_dl = b.take<double>(E); d.hy_g = b.take<double>(E); d.hy_phi = b.take<double>(E);
    }
    d.red_stride = (int32_t)(((N + kBlock - 1) / kBlock + 7) / 8 * 8);
    d.red_stride2 = (d.red_stride + kGroup - 1) / kGroup;
    d.partials = b.take<double>((size_t)kMaxRed * d.red_stride);
    d.partials2 = b.take<double>((size_t)kMaxRed * d.red_stride2);
    d.gticket = b.take<unsigned int>((size_t)d.red_stride2);
    d.ticket = b.take<unsigned int>(64);
    d.ks = b.take<KState>(kNumKs);
    d.ks_gather = b.take<KState>((size_t)kMaxBatch * kNumKs);
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
    if (o->p_ctl.precond != FVM_PC_JACOBI && o->p_ctl.precond != FVM_PC_DIC && o->p_ctl.precond != FVM_PC_AMG)
        return fvm_fail(FVM_EINVAL, "case: bad preconditioner");
    if (o->precision == FVM_MIXED && o->p_ctl.precond == FVM_PC_AMG)
        return fvm_fail(FVM_EINVAL, "case: the AMG preconditioner is FP64 only");
    if (o->u_ctl.precond != FVM_PC_JACOBI) return fvm_fail(FVM_EINVAL, "case: momentum solver takes Jacobi only");
    if (o->p_ctl.max_iter < 1 || o->u_ctl.max_iter < 1) return fvm_fail(FVM_EINVAL, "case: max_iter must be >= 1");
    if (!(o->p_ctl.tol >= 0.0) || !(o->u_ctl.tol >= 0.0) || !(o->p_ctl.rel_tol >= 0.0) || !(o->u_ctl.rel_tol >= 0.0))
        return fvm_fail(FVM_EINVAL, "case: tolerances must be >= 0");
    if (o->convection != FVM_CONV_LINEAR && o->convection != FVM_CONV_UPWIND)
        return fvm_fail(FVM_EINVAL, "case: bad convection scheme");
    if (o->u_solver != FVM_SOLVER_BICG && o->u_solver != FVM_SOLVER_BICGSTAB)
        return fvm_fail(FVM_EINVAL, "case: bad momentum solver");
    if (o->u_solver == FVM_SOLVER_BICGSTAB && o->precision != FVM_FP64)
        return fvm_fail(FVM_EINVAL, "case: the BiCGStab momentum solver is FP64 only");
    if (o->hybrid_K < 0 || o->hybrid_K > 64) return fvm_fail(FVM_EINVAL, "case: hybrid_K must be in [0, 64]");
    if (o->hybrid_K > 0 && (int64_t)o->hybrid_K * m->N >= INT32_MAX)
        return fvm_fail(FVM_EINVAL, "case: hybrid_K * n_cells exceeds int32");
    if (o->step_kernel != FVM_STEP_AUTO && o->step_kernel != FVM_STEP_LAUNCHED)
        return fvm_fail(FVM_EINVAL, "case: bad step_kernel");
    return FVM_OK;
}

constexpr int kRing = 4;

// Pinned ring of Krylov-state copies (kMaxBatch cases x kNumKs states per
// slot) with one event per slot: the host inspects the copy of chunk k while
// chunk k+1 runs.
struct Poller {
    KState *h = nullptr;
    hipEvent_t ev[kRing];
    bool pending[kRing] = {false, false, false, false};
    int ring = 0;
    bool ok = false;
    fvm_status init()
    {
        if (ok) return FVM_OK;
        const hipError_t e = hipHostMalloc((void **)&h, sizeof(KState) * kMaxBatch * kNumKs * kRing, hipHostMallocDefault);
        if (e != hipSuccess) return fvm_fail(FVM_EDEVICE, std::string("poller: pinned host buffer: ") + hipGetErrorString(e));
        for (int k = 0; k < kRing; ++k)
            if (hipEventCreateWithFlags(&ev[k], hipEventDisableTiming) != hipSuccess)
                return fvm_fail(FVM_EDEVICE, "poller: event");
        ok = true;
        return FVM_OK;
    }
    void release()
    {
        if (!ok) return;
        for (int k = 0; k < kRing; ++k) {
            if (pending[k]) (void)hipEventSynchronize(ev[k]);
            (void)hipEventDestroy(ev[k]);
        }
        (void)hipHostFree(h);
        ok = false;
    }
    KState *slot_ptr(int slot) { return h + (size_t)slot * kMaxBatch * kNumKs; }
};

}  // namespace

struct fvm_case {
    fvm_case_opts o;
    DevCase d;                      // host copy; d.self is the device copy
    int32_t N, F, Fi, Fb, npatch;
    bool nonorth, has_fixed_p;
    std::vector<fvm_patch> patches;
    Poller poll;
    int last_iters[4] = {0, 0, 0, 0};   // momentum, pressure, momentum inner; chunk sizing
    // whole PISO steps in one workgroup (see FVM_STEP_AUTO)
    bool solo() const
    {
        return o.step_kernel == FVM_STEP_AUTO && N <= kSoloMaxCells && !nonorth && o.n_non_orth_corr == 0 &&
               o.n_corr <= kSoloMaxCorr && o.p_ctl.precond == FVM_PC_JACOBI && o.u_solver == FVM_SOLVER_BICG;
    }
};

namespace {

// a group of resident cases advanced by shared launches
// Captured chunks of Krylov iterations.  The descriptor table of a group is
// a kernel argument that stays fixed while the group exists, so a chunk of
// kGraphIters iterations of one solve kind is captured once per group and
// then launched as one graph (one submission instead of 3-5 per iteration);
// iterations past the last whole chunk are launched directly.  Every
// captured node is a kernel launch.
constexpr int kGraphIters = 8;
constexpr int kGraphKinds = 8;
struct GraphCache {
    hipGraphExec_t ex[kGraphKinds] = {};
    bool failed[kGraphKinds] = {};
    GraphCache() = default;
    GraphCache(const GraphCache &) = delete;
    GraphCache &operator=(const GraphCache &) = delete;
    ~GraphCache()
    {
        for (auto &e : ex)
            if (e) (void)hipGraphExecDestroy(e);
    }
};

// a non-blocking stream of the current device to capture on (capture is
// not possible on the legacy default stream a caller may pass)
hipStream_t capture_stream()
{
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return nullptr;
    static thread_local hipStream_t cs[64] = {};
    if (!cs[dev] && hipStreamCreateWithFlags(&cs[dev], hipStreamNonBlocking) != hipSuccess) cs[dev] = nullptr;
    return cs[dev];
}

struct Group {
    std::vector<fvm_case *> cs;
    BatchSet bs;
    Poller *poll;
    hipStream_t s;
    std::shared_ptr<GraphCache> graphs = std::make_shared<GraphCache>();
    explicit Group(fvm_case *c, hipStream_t st) : poll(&c->poll), s(st)
    {
        cs.push_back(c);
        bs.n = 0;
        batch_add(bs, c->d.self, &c->d);
    }
    Group(fvm_case *const *c, int n, Poller *p, hipStream_t st) : poll(p), s(st)
    {
        bs.n = 0;
        for (int i = 0; i < n; ++i) {
            cs.push_back(c[i]);
            batch_add(bs, c[i]->d.self, &c[i]->d);
        }
    }
    int n() const { return (int)cs.size(); }
};

thread_local Poller t_batch_poll;

}  // namespace

namespace {
// a roctx range over one phase of the host driver (momentum assembly and
// solve, pressure assembly and solve, corrections, whole steps): rocprofv3
// --marker-trace shows where a step's time goes; without a tool attached a
// range costs a function call
struct Phase {
    explicit Phase(const char *name) { roctxRangePushA(name); }
    ~Phase() { roctxRangePop(); }
    Phase(const Phase &) = delete;
    Phase &operator=(const Phase &) = delete;
};
}  // namespace

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
    if (bytes < need)
        return fvm_fail(FVM_ENOMEM, "case: workspace too small (" + std::to_string(bytes) + " < " + std::to_string(need) + ")");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    fvm_case *c = new (std::nothrow) fvm_case();
    if (!c) return fvm_fail(FVM_ENOMEM, "case: out of host memory");
    c->o = *o;
    c->N = m->N; c->F = m->F; c->Fi = m->Fi; c->Fb = m->Fb; c->npatch = m->npatch;
    c->nonorth = m->nonorth; c->has_fixed_p = m->has_fixed_p;
    c->patches = m->patches;
    Bump b{reinterpret_cast<char *>(ws)};
    std::vector<AmgLevel> amg_lv;
    plan(*m, *o, b, c->d, &amg_lv);
    auto fail = [&](fvm_status code) {
        c->poll.release();
        delete c;
        return code;
    };
    st = c->poll.init();
    if (st != FVM_OK) return fail(st);
    DevCase &d = c->d;
    const int np = c->npatch;
    std::vector<int32_t> uk(np), pk(np);
    std::vector<int32_t> smode = m->sell_mode;   // uploaded below; alive until the final synchronisation
    std::vector<double> uv(3 * (size_t)np), pv(np);
    for (int p = 0; p < np; ++p) {
        uk[p] = c->patches[p].u_kind; pk[p] = c->patches[p].p_kind; pv[p] = c->patches[p].p_value;
        for (int k = 0; k < 3; ++k) uv[3 * p + k] = c->patches[p].u_value[k];
    }
    const size_t F = m->F;
#define UPCHK(x) do { if ((x) != hipSuccess) return fail(fvm_fail(FVM_EDEVICE, "case: upload " #x)); } while (0)
    UPCHK(hipMemcpyAsync(d.self, &c->d, sizeof(DevCase), hipMemcpyHostToDevice, s));
    UPCHK(up(d.own, m->own, s)); UPCHK(up(d.nei, m->nei, s));
    UPCHK(up(d.own_start, m->own_start, s)); UPCHK(up(d.nbr_start, m->nbr_start, s)); UPCHK(up(d.losort, m->losort, s));
    UPCHK(up(d.bnd_start, m->bnd_start, s)); UPCHK(up(d.bnd_list, m->bnd_list, s)); UPCHK(up(d.bpatch, m->bpatch, s));
    UPCHK(up(d.face_user, m->face_user, s)); UPCHK(up(d.face_sign, m->face_sign, s));
    UPCHK(up(d.patch_uk, uk, s)); UPCHK(up(d.patch_pk, pk, s)); UPCHK(up(d.patch_uv, uv, s)); UPCHK(up(d.patch_pv, pv, s));
    UPCHK(hipMemcpyAsync(d.Sx, m->S.data(), sizeof(double) * F, hipMemcpyHostToDevice, s));
    UPCHK(hipMemcpyAsync(d.Sy, m->S.data() + F, sizeof(double) * F, hipMemcpyHostToDevice, s));
    UPCHK(hipMemcpyAsync(d.Sz, m->S.data() + 2 * F, sizeof(double) * F, hipMemcpyHostToDevice, s));
    UPCHK(up(d.V, m->V, s));
    UPCHK(up(d.tmpC, m->C, s));
    UPCHK(up(d.tmpCf, m->Cf, s));
    if (d.lvl_cells) {
        UPCHK(up(d.lvl_cells, m->lvl_cells, s));
        UPCHK(up(d.dl_pos, m->dl_pos, s)); UPCHK(up(d.dl_face, m->dl_face, s));
        UPCHK(up(d.du_pos, m->du_pos, s)); UPCHK(up(d.du_face, m->du_face, s));
    }
    {
        // a regular slice none of whose cells has a fixed-pressure face or
        // the reference pin has each diagonal equal to minus the sum of its
        // row's coefficients (mode 2: the product derives it)
        std::vector<int32_t> &mode = smode;
        const int32_t ns = (int32_t)mode.size();
        for (int32_t sl = 0; sl < ns; ++sl) {
            if (mode[sl] != 0) continue;
            bool plain = true;
            const int32_t i0 = sl * kBlock, i1 = std::min(m->N, i0 + kBlock);
            for (int32_t i = i0; i < i1 && plain; ++i) {
                if (i == o->p_ref_cell && !m->has_fixed_p) plain = false;
                for (int32_t k = m->bnd_start[i]; k < m->bnd_start[i + 1] && plain; ++k)
                    plain = pk[m->bpatch[m->bnd_list[k]]] != FVM_BC_FIXED;
            }
            if (plain) mode[sl] = 2;
        }
        UPCHK(up(d.sell_mode, mode, s));
    }
    UPCHK(up(d.sell_off, m->sell_off, s)); UPCHK(up(d.sell_mir, m->sell_mir, s));
    UPCHK(up(d.sell_fe, m->sell_fe, s)); UPCHK(up(d.sell_col, m->sell_col, s));
    if (d.amg_nl > 0) {
        const AmgHost &A = mesh_amg(*m);
        if (d.amg_nc > kAmgDenseMax)
            return fail(fvm_fail(FVM_EINVAL, "case: AMG coarsening stalled above the dense coarsest size"));
        auto w = [](const int32_t *p) { return const_cast<int32_t *>(p); };
        for (int l = 0; l < d.amg_nl; ++l) {
            const AmgLevelHost &L = A.L[l];
            const AmgLevel &e = amg_lv[l];
            if (l > 0) {
                UPCHK(up(w(e.own), L.own, s)); UPCHK(up(w(e.nei), L.nei, s));
                UPCHK(up(w(e.own_start), L.own_start, s)); UPCHK(up(w(e.nbr_start), L.nbr_start, s));
                UPCHK(up(w(e.losort), L.losort, s));
                UPCHK(up(w(e.mstart), L.mstart, s)); UPCHK(up(w(e.members), L.members, s));
                UPCHK(up(w(e.istart), L.istart, s)); UPCHK(up(w(e.inner), L.inner, s));
                UPCHK(up(w(e.cstart), L.cstart, s)); UPCHK(up(w(e.cfaces), L.cfaces, s));
            }
            if (l < d.amg_nl - 1) UPCHK(up(w(e.agg), L.agg, s));
        }
        UPCHK(hipMemcpyAsync(d.amg, amg_lv.data(), sizeof(AmgLevel) * amg_lv.size(), hipMemcpyHostToDevice, s));
    }
    HybridHost hy;
    if (d.hy_K > 0) {
        build_hybrid(*m, d.hy_K, hy);
        if (hy.nC != d.hy_nC || (int64_t)d.hy_K * m->N + hy.nC >= INT32_MAX)
            return fail(fvm_fail(FVM_EINVAL, "case: hybrid layout too large for int32 positions"));
        UPCHK(up(d.hy_I, hy.dI, s)); UPCHK(up(d.hy_J, hy.dJ, s)); UPCHK(up(d.hy_dpos, hy.dpos, s));
        UPCHK(up(d.hy_locO, hy.locO, s)); UPCHK(up(d.hy_locN, hy.locN, s));
        UPCHK(up(d.hy_cstart, hy.c_start, s)); UPCHK(up(d.hy_ccol, hy.c_col, s)); UPCHK(up(d.hy_ctrpos, hy.c_trpos, s));
        const size_t E = (size_t)d.hy_K * m->N + hy.nC;
        for (double *a : {d.hy_V, d.hy_Sx, d.hy_Sy, d.hy_Sz, d.hy_w, d.hy_dl, d.hy_g, d.hy_phi})
            UPCHK(hipMemsetAsync(a, 0, E * sizeof(double), s));
    }
    UPCHK(hipMemsetAsync(d.ticket, 0, 64 * sizeof(unsigned int), s));
    UPCHK(hipMemsetAsync(d.gticket, 0, d.red_stride2 * sizeof(unsigned int), s));
    UPCHK(hipMemsetAsync(d.ks, 0, kNumKs * sizeof(KState), s));
    const Group g(c, s);
    launch_init_partials(g.bs, s);
    launch_geometry(g.bs, s);
    if (d.hy_K > 0) launch_hybrid_geometry(g.bs, s);
    UPCHK(hipMemsetAsync(d.U, 0, 3 * (size_t)m->N * sizeof(double), s));
    UPCHK(hipMemsetAsync(d.p, 0, (size_t)m->N * sizeof(double), s));
    launch_flux_from_U(g.bs, s);
    UPCHK(hipGetLastError());
    UPCHK(hipStreamSynchronize(s));   // host vectors above are temporaries
#undef UPCHK
    *out = c;
    return FVM_OK;
}

extern "C" void fvm_case_destroy(fvm_case *c)
{
    if (!c) return;
    c->poll.release();
    delete c;
}

// ---------------------------------------------------------------------------
// public: state exchange
// ---------------------------------------------------------------------------
extern "C" fvm_status fvm_case_set_state(fvm_case *c, const double *U, const double *p, const double *phi, void *stream)
{
    if (!c) return fvm_fail(FVM_EINVAL, "case: null handle");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const Group g(c, s);
    if (U) launch_U_in(g.bs, U, s);
    if (p) HIPCHK(hipMemcpyAsync(c->d.p, p, sizeof(double) * c->N, hipMemcpyDeviceToDevice, s));
    if (phi) launch_phi_in(g.bs, phi, s);
    else launch_flux_from_U(g.bs, s);
    HIPCHK(hipGetLastError());
    return FVM_OK;
}

extern "C" fvm_status fvm_case_get_state(const fvm_case *c, double *U, double *p, double *phi, void *stream)
{
    if (!c) return fvm_fail(FVM_EINVAL, "case: null handle");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const Group g(const_cast<fvm_case *>(c), s);
    if (U) launch_U_out(g.bs, U, s);
    if (p) HIPCHK(hipMemcpyAsync(p, c->d.p, sizeof(double) * c->N, hipMemcpyDeviceToDevice, s));
    if (phi) launch_phi_out(g.bs, phi, s);
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
    const Group g(c, s);
    launch_set_patch(g.bs, patch, u_value[0], u_value[1], u_value[2], p_value, s);
    HIPCHK(hipGetLastError());
    return FVM_OK;
}

// ---------------------------------------------------------------------------
// Krylov drivers (over a group of cases)
// ---------------------------------------------------------------------------
namespace {

// copy every case's states into the poller slot (one gather kernel + one
// D2H copy); returns the slot index
fvm_status enqueue_states(Group &g, int &slot_out)
{
    Poller &P = *g.poll;
    const int slot = P.ring;
    P.ring = (P.ring + 1) % kRing;
    if (P.pending[slot]) {
        HIPCHK(hipEventSynchronize(P.ev[slot]));
        P.pending[slot] = false;
    }
    const DevCase &lead = g.cs[0]->d;
    if (g.n() == 1) {
        HIPCHK(hipMemcpyAsync(P.slot_ptr(slot), lead.ks, kNumKs * sizeof(KState), hipMemcpyDeviceToHost, g.s));
    } else {
        launch_gather_ks(g.bs, g.s);
        HIPCHK(hipMemcpyAsync(P.slot_ptr(slot), lead.ks_gather, (size_t)g.n() * kNumKs * sizeof(KState),
                              hipMemcpyDeviceToHost, g.s));
    }
    HIPCHK(hipEventRecord(P.ev[slot], g.s));
    P.pending[slot] = true;
    slot_out = slot;
    return FVM_OK;
}

fvm_status wait_slot(Group &g, int slot)
{
    HIPCHK(hipEventSynchronize(g.poll->ev[slot]));
    g.poll->pending[slot] = false;
    return FVM_OK;
}

// state k of case i in a slot
inline const KState &st_of(Group &g, int slot, int i, int k) { return g.poll->slot_ptr(slot)[(size_t)i * kNumKs + k]; }

// Enqueue iterations in chunks until the systems [first, first+count) of
// every case are finished (done == 1; 2 means paused for a device-side
// check); res[i*kNumKs + k] receives the final states.  launch_iter(stream,
// k) enqueues iteration k (counted from 0) on the stream; `predicted` sizes
// the first chunk.  gkey (0 <= gkey < kGraphKinds) names the solve kind for
// captured chunks (-1: never capture); the enqueued work does not depend on
// whether a chunk was captured.  No capture while per-launch profiling
// events are being recorded.
bool prof_active() { return g_prof_on; }

template <class F>
fvm_status iterate_until_done(Group &g, int first, int count, int predicted, long limit, int gkey, F launch_iter,
                              std::vector<KState> &res)
{
    int chunk = predicted > 0 ? std::max(2, predicted - predicted / 4) : 4;
    long issued = 0;
    int prev = -1;
    auto all_done = [&](int slot) {
        for (int i = 0; i < g.n(); ++i)
            for (int k = 0; k < count; ++k)
                if (st_of(g, slot, i, first + k).done != 1) return false;
        return true;
    };
    auto take = [&](int slot) {
        res.assign(g.poll->slot_ptr(slot), g.poll->slot_ptr(slot) + (size_t)g.n() * kNumKs);
    };
    GraphCache &gc = *g.graphs;
    const bool graphs_ok = gkey >= 0 && gkey < kGraphKinds && !prof_active();
    // the captured chunk (built on first use; a failure turns capture off
    // for this kind and the iterations are launched directly)
    auto graph = [&]() -> hipGraphExec_t {
        if (!graphs_ok || gc.failed[gkey]) return nullptr;
        if (gc.ex[gkey]) return gc.ex[gkey];
        hipStream_t cs = capture_stream();
        hipGraph_t gr = nullptr;
        hipGraphExec_t ex = nullptr;
        bool ok = cs && hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess;
        if (ok) {
            for (int k = 0; k < kGraphIters; ++k) launch_iter(cs, k);
            ok = hipStreamEndCapture(cs, &gr) == hipSuccess && gr;
        }
        if (ok) ok = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0) == hipSuccess;
        if (gr) (void)hipGraphDestroy(gr);
        (void)hipGetLastError();
        if (!ok) {
            gc.failed[gkey] = true;
            return nullptr;
        }
        gc.ex[gkey] = ex;
        return ex;
    };
    for (;;) {
        const long n = std::min<long>(chunk, std::max<long>(1, limit - issued));
        long done_n = 0;
        while (done_n < n) {
            hipGraphExec_t ex = (issued % kGraphIters == 0 && n - done_n >= kGraphIters) ? graph() : nullptr;
            if (ex) {
                HIPCHK(hipGraphLaunch(ex, g.s));
                issued += kGraphIters;
                done_n += kGraphIters;
            } else {
                launch_iter(g.s, issued);
                ++issued;
                ++done_n;
            }
        }
        HIPCHK(hipGetLastError());
        int slot;
        fvm_status st = enqueue_states(g, slot);
        if (st != FVM_OK) return st;
        if (prev >= 0) {
            st = wait_slot(g, prev);
            if (st != FVM_OK) return st;
            if (all_done(prev)) {
                take(prev);
                return FVM_OK;
            }
        }
        if (issued >= limit) {
            st = wait_slot(g, slot);
            if (st != FVM_OK) return st;
            if (!all_done(slot)) return fvm_fail(FVM_EDEVICE, "solve: iteration limit passed without a stop flag");
            take(slot);
            return FVM_OK;
        }
        prev = slot;
        // later chunks stay short: the launches enqueued past the stop flag
        // (up to two chunks) return at once but still cost a launch each
        chunk = predicted > 0 ? std::min(64, std::max(2, predicted / 8)) : std::min(64, chunk * 2);
    }
}

fvm_status snapshot(Group &g, std::vector<KState> &res)
{
    int slot;
    fvm_status st = enqueue_states(g, slot);
    if (st != FVM_OK) return st;
    st = wait_slot(g, slot);
    if (st != FVM_OK) return st;
    res.assign(g.poll->slot_ptr(slot), g.poll->slot_ptr(slot) + (size_t)g.n() * kNumKs);
    return FVM_OK;
}

int predicted_iters(Group &g, int slot)
{
    int m = 0;
    for (auto *c : g.cs) m = std::max(m, c->last_iters[slot]);
    return m;
}

void record_iters(Group &g, const std::vector<KState> &res, int first, int count, int slot)
{
    for (int i = 0; i < g.n(); ++i) {
        int m = 0;
        for (int k = 0; k < count; ++k) m = std::max(m, res[(size_t)i * kNumKs + first + k].iters);
        g.cs[i]->last_iters[slot] = m;
    }
}

// One solve for every case of the group.  kind 0: momentum BiCG (systems
// 0..2), kind 1: pressure CG (system 3).  ctl_src selects the controls:
// 0/1 = the cases' own momentum / pressure controls, 2 = *ctl.
// FVM_MIXED cases run the mixed-precision variants.
fvm_status run_solve(Group &g, int kind, int ctl_src, const fvm_solver_ctl *ctl, std::vector<KState> &res)
{
    const BatchSet &bs = g.bs;
    hipStream_t s = g.s;
    fvm_case *c0 = g.cs[0];
    const int first = kind == 0 ? 0 : 3, count = kind == 0 ? 3 : 1;
    const int precond = ctl_src == 2 ? ctl->precond : c0->o.p_ctl.precond;
    const int dic = kind == 1 && precond == FVM_PC_DIC;
    const int amg = kind == 1 && precond == FVM_PC_AMG;
    const int pc = dic ? 1 : amg ? 2 : 0;     // external preconditioner (z and rho from it)
    const bool mixed = c0->o.precision == FVM_MIXED;
    long max_iter = 0;
    for (auto *c : g.cs)
        max_iter = std::max<long>(max_iter, ctl_src == 2 ? ctl->max_iter : kind == 0 ? c->o.u_ctl.max_iter : c->o.p_ctl.max_iter);
    launch_set_ctl(bs, first, count, ctl_src, ctl ? ctl->tol : 0.0, ctl ? ctl->rel_tol : 0.0, ctl ? ctl->max_iter : 0, s);
    if (kind == 0) launch_bicg_init(bs, c0->o.u_solver == FVM_SOLVER_BICGSTAB, s);
    else launch_pcg_init(bs, pc, s);
    fvm_status st;
    if (!mixed) {
        if (dic) launch_dic_precond(bs, 1, s);
        else if (amg) launch_amg_precond(bs, 1, s);
        const bool stab = kind == 0 && c0->o.u_solver == FVM_SOLVER_BICGSTAB;
        const int gkey = stab ? 2 : kind == 0 ? 0 : (dic ? 3 : amg ? 6 : 1);
        st = iterate_until_done(g, first, count, predicted_iters(g, kind), max_iter + 1, gkey, [&](hipStream_t st_, long k) {
            if (stab) launch_bicgstab_iter(bs, st_);
            else if (kind == 0) launch_bicg_iter(bs, st_);
            else launch_pcg_iter(bs, pc, (int)(k & 1), st_);
        }, res);
        if (st != FVM_OK) return st;
    } else if (kind == 1) {
        // FP32 CG recurrence, FP64 solution; the replacement kernel follows
        // every kReplaceEvery-th iteration and does nothing unless the device
        // state asks for a replacement (paused at the tolerance or the
        // iteration limit, or the recurrence residual fell 10x since the last
        // one).  Iterations enqueued while paused are no-ops, so the launch
        // limit is a multiple of max_iter; the device enforces max_iter.
        constexpr int kReplaceEvery = 4;
        static_assert(kGraphIters % kReplaceEvery == 0, "captured chunks must repeat the replacement pattern");
        launch_rr_start(bs, s);
        st = iterate_until_done(g, first, count, predicted_iters(g, kind), (max_iter + 2) * kReplaceEvery, 4,
                                [&](hipStream_t st_, long k) {
                                    launch_rr_iter(bs, (int)(k & 1), st_);
                                    if ((k + 1) % kReplaceEvery == 0) launch_rr_replace(bs, st_);
                                }, res);
        if (st != FVM_OK) return st;
    } else {
        // momentum: FP64 refinement around restarted FP32 BiCG solves
        long inner_max = 0;
        for (auto *c : g.cs) inner_max = std::max<long>(inner_max, c->o.inner_max_iter);
        launch_set_ctl(bs, 4, 3, 3, 0.0, 0.0, 0, s);
        launch_mx_cvt(bs, 0, s);
        for (int outer = 0;; ++outer) {
            st = snapshot(g, res);
            if (st != FVM_OK) return st;
            bool all = true;
            for (int i = 0; i < g.n(); ++i)
                for (int k = 0; k < 3; ++k) all = all && res[(size_t)i * kNumKs + k].done == 1;
            if (all) break;
            if (outer >= 1000) return fvm_fail(FVM_EDEVICE, "solve: refinement did not terminate");
            launch_mx_inner_init(bs, 0, s);
            st = iterate_until_done(g, 4, 3, predicted_iters(g, 2), inner_max + 1, 5,
                                    [&](hipStream_t st_, long) { launch_mx_inner_iter(bs, 0, st_); }, res);
            if (st != FVM_OK) return st;
            record_iters(g, res, 4, 3, 2);
            launch_mx_correct_resid(bs, 0, s);
        }
        // components whose FP32 inner solve broke down continue as FP64
        // BiCG solves from their current iterate
        bool fb = false;
        for (int i = 0; i < g.n(); ++i)
            for (int k = 0; k < 3; ++k) fb = fb || res[(size_t)i * kNumKs + k].status == kStatusFallback;
        if (fb) {
            launch_bicg_fallback(bs, s);
            st = iterate_until_done(g, 0, 3, predicted_iters(g, kind), max_iter + 1, 0,
                                    [&](hipStream_t st_, long) { launch_bicg_iter(bs, st_); }, res);
            if (st != FVM_OK) return st;
        }
    }
    record_iters(g, res, first, count, kind);
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

// momentum matrix + predictor solve; mode 0 PISO, 1 SIMPLE
fvm_status momentum_predictor(Group &g, int mode, std::vector<fvm_step_info> &info)
{
    {
        Phase ph("momentum assembly");
        launch_gradU(g.bs, g.s);
        launch_mom_face(g.bs, g.s);
        launch_mom_cell(g.bs, mode, g.s);
    }
    std::vector<KState> res;
    fvm_status st;
    {
        Phase ph("momentum solve");
        st = run_solve(g, 0, 0, nullptr, res);
    }
    if (st != FVM_OK) return st;
    for (int i = 0; i < g.n(); ++i)
        for (int k = 0; k < 3; ++k) {
            to_info(res[(size_t)i * kNumKs + k], info[i].u[k]);
            worst(info[i].status, res[(size_t)i * kNumKs + k].status);
        }
    return FVM_OK;
}

fvm_status pressure_solve(Group &g, std::vector<fvm_step_info> &info)
{
    std::vector<KState> res;
    fvm_status st;
    {
        Phase ph("pressure solve");
        st = run_solve(g, 1, 1, nullptr, res);
    }
    if (st != FVM_OK) return st;
    for (int i = 0; i < g.n(); ++i) {
        const KState &k = res[(size_t)i * kNumKs + 3];
        if (info[i].n_p_solves < 16) to_info(k, info[i].p[info[i].n_p_solves++]);
        worst(info[i].status, k.status);
    }
    return FVM_OK;
}

bool any_failed(const std::vector<fvm_step_info> &info)
{
    for (auto &i : info)
        if (i.status < 0) return true;
    return false;
}

// one PISO step of every case of the group; a case whose solve failed keeps
// going (its kernels see non-finite values) and is rolled back afterwards
fvm_status piso_one(Group &g, std::vector<fvm_step_info> &info)
{
    info.assign(g.n(), fvm_step_info{});
    fvm_status st = momentum_predictor(g, 0, info);
    if (st != FVM_OK) return st;
    const fvm_case *c0 = g.cs[0];
    if (!(g.n() == 1 && any_failed(info)))
        for (int corr = 0; corr < c0->o.n_corr; ++corr) {
            for (int k = 0; k <= c0->o.n_non_orth_corr; ++k) {
                {
                    Phase ph("pressure assembly");
                    if (k == 0) launch_hbya(g.bs, 1, g.s);
                    else launch_gradp(g.bs, g.s);
                    launch_p_face(g.bs, g.s);
                    launch_p_cell(g.bs, g.s);
                }
                st = pressure_solve(g, info);
                if (st != FVM_OK) return st;
                if (g.n() == 1 && any_failed(info)) return FVM_OK;
            }
            Phase ph("corrections");
            launch_flux_corr(g.bs, g.s);
            launch_U_corr(g.bs, g.s);
        }
    HIPCHK(hipGetLastError());
    return FVM_OK;
}

fvm_status simple_one(Group &g, std::vector<fvm_step_info> &info)
{
    info.assign(g.n(), fvm_step_info{});
    fvm_status st = momentum_predictor(g, 1, info);
    if (st != FVM_OK || any_failed(info)) return st;
    {
        Phase ph("pressure assembly");
        for (auto *c : g.cs)
            HIPCHK(hipMemcpyAsync(c->d.p_prev, c->d.p, sizeof(double) * c->N, hipMemcpyDeviceToDevice, g.s));
        launch_hbya(g.bs, 1, g.s);
        launch_p_face(g.bs, g.s);
        launch_p_cell(g.bs, g.s);
    }
    st = pressure_solve(g, info);
    if (st != FVM_OK || any_failed(info)) return st;
    Phase ph("corrections");
    launch_flux_corr(g.bs, g.s);
    launch_p_relax(g.bs, g.s);
    launch_U_corr(g.bs, g.s);
    HIPCHK(hipGetLastError());
    return FVM_OK;
}

// roll back the cases of the group whose step failed
fvm_status rollback_failed(Group &g, const std::vector<fvm_step_info> &info)
{
    for (int i = 0; i < g.n(); ++i)
        if (info[i].status < 0) {
            const Group one(g.cs[i], g.s);
            launch_save(one.bs, 1, g.s);
        }
    HIPCHK(hipStreamSynchronize(g.s));
    return FVM_OK;
}

}  // namespace

// ---------------------------------------------------------------------------
// public: PISO, SIMPLE, stand-alone pressure solve, batch
// ---------------------------------------------------------------------------
namespace {
// n_steps PISO steps of every case of the group in one launch, one
// workgroup per case; the kernel leaves each case's last-step record in its
// Krylov state slots: 0..2 momentum, 3.. the pressure solves, the last one a
// summary (iters: pressure solves recorded, status: worst over the steps,
// done: steps completed, first: 1 when a step failed and was rolled back)
fvm_status piso_solo(Group &g, int32_t n_steps, fvm_step_info *infos)
{
    const int n = g.n();
    Phase ph("whole-step launch");
    if (n_steps > 0) launch_solo_piso(g.bs, n_steps, g.cs[0]->o.n_corr, g.s);
    HIPCHK(hipGetLastError());
    std::vector<KState> res;
    int32_t all = FVM_OK;
    if (n_steps > 0) {
        fvm_status st = snapshot(g, res);
        if (st != FVM_OK) return st;
    }
    bool failed = false;
    for (int i = 0; i < n; ++i) {
        fvm_step_info info{};
        if (n_steps > 0) {
            const KState *r = res.data() + (size_t)i * kNumKs;
            const KState &m = r[kNumKs - 1];
            for (int c = 0; c < 3; ++c) {
                to_info(r[c], info.u[c]);
                worst(info.status, r[c].status);
            }
            info.n_p_solves = std::min(m.iters, kNumKs - 4);
            for (int k = 0; k < info.n_p_solves; ++k) {
                to_info(r[3 + k], info.p[k]);
                worst(info.status, r[3 + k].status);
            }
            worst(all, m.status);
            failed = failed || m.first != 0;
            int32_t &li = g.cs[i]->last_iters[1];
            li = info.n_p_solves > 0 ? info.p[info.n_p_solves - 1].iters : li;
        }
        if (infos) infos[i] = info;
    }
    if (all < 0 || failed)
        return fvm_fail(all < 0 ? all : FVM_ENUMERIC,
                        "piso: a solve failed (non-finite value or breakdown); the case was rolled back");
    return all;
}
}  // namespace

extern "C" fvm_status piso_step(fvm_case *c, int32_t n_steps, void *stream, fvm_step_info *last)
{
    if (!c) return fvm_fail(FVM_EINVAL, "piso: null handle");
    return piso_step_batch(&c, 1, n_steps, stream, last);
}

extern "C" fvm_status simple_iterate(fvm_case *c, int32_t max_iters, double res_tol, void *stream, int32_t *iters_done,
                                     fvm_step_info *last)
{
    if (!c) return fvm_fail(FVM_EINVAL, "simple: null handle");
    if (max_iters < 0) return fvm_fail(FVM_EINVAL, "simple: max_iters < 0");
    if (!(c->o.alpha_u > 0.0 && c->o.alpha_u <= 1.0) || !(c->o.alpha_p > 0.0 && c->o.alpha_p <= 1.0))
        return fvm_fail(FVM_EINVAL, "simple: relaxation factors must be in (0, 1]");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Group g(c, s);
    int32_t acc = FVM_OK, it = 0;
    std::vector<fvm_step_info> info(1, fvm_step_info{});
    for (it = 0; it < max_iters;) {
        Phase ph("simple iteration");
        launch_save(g.bs, 0, s);
        fvm_status st = simple_one(g, info);
        if (st != FVM_OK) return st;
        if (info[0].status < 0) {
            rollback_failed(g, info);
            if (iters_done) *iters_done = it;
            if (last) *last = info[0];
            return fvm_fail(info[0].status, "simple: a solve failed (non-finite value or breakdown)");
        }
        ++it;
        worst(acc, info[0].status);
        if (info[0].u[0].res_initial <= res_tol && info[0].u[1].res_initial <= res_tol &&
            info[0].u[2].res_initial <= res_tol && info[0].p[0].res_initial <= res_tol)
            break;
    }
    if (last) HIPCHK(hipStreamSynchronize(s));
    if (iters_done) *iters_done = it;
    if (last) *last = info[0];
    return acc;
}

extern "C" fvm_status solve_pressure(fvm_case *c, const double *gamma, const double *rhs, double *p,
                                     const fvm_solver_ctl *ctl, void *stream, fvm_solve_info *out)
{
    if (!c || !gamma || !rhs || !p || !ctl) return fvm_fail(FVM_EINVAL, "solve_pressure: null argument");
    if (ctl->precond != FVM_PC_JACOBI && ctl->precond != FVM_PC_DIC && ctl->precond != FVM_PC_AMG)
        return fvm_fail(FVM_EINVAL, "solve_pressure: bad preconditioner");
    if (ctl->precond == FVM_PC_DIC && !c->d.dstar)
        return fvm_fail(FVM_EINVAL, "solve_pressure: DIC needs a case created with the DIC preconditioner");
    if (ctl->precond == FVM_PC_AMG && c->d.amg_nl < 1)
        return fvm_fail(FVM_EINVAL, "solve_pressure: AMG needs a case created with the AMG preconditioner");
    if (ctl->max_iter < 1) return fvm_fail(FVM_EINVAL, "solve_pressure: max_iter must be >= 1");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Group g(c, s);
    const DevCase &d = c->d;
    // the case's p field is the solver's unknown: park it
    HIPCHK(hipMemcpyAsync(d.p_save, d.p, sizeof(double) * c->N, hipMemcpyDeviceToDevice, s));
    launch_gather_faces(g.bs, gamma, d.phiH, s);
    launch_p_system_from_gamma(g.bs, d.phiH, rhs, s);
    HIPCHK(hipMemcpyAsync(d.p, p, sizeof(double) * c->N, hipMemcpyDeviceToDevice, s));
    std::vector<KState> res;
    fvm_status st = run_solve(g, 1, 2, ctl, res);
    if (st != FVM_OK) return st;
    const KState &ks = res[3];
    if (ks.status >= 0) HIPCHK(hipMemcpyAsync(p, d.p, sizeof(double) * c->N, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(d.p, d.p_save, sizeof(double) * c->N, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    if (out) to_info(ks, *out);
    if (ks.status < 0) return fvm_fail(ks.status, "solve_pressure: non-finite value or breakdown");
    return ks.status;
}

namespace {
// bytes of the static scratch a case's reduction slots, tickets, Krylov
// states and descriptor copy take (256-byte aligned sections)
size_t static_layout(const DevCase &d, DevCase *h, unsigned char *base)
{
    size_t off = 0;
    auto take = [&](size_t bytes) {
        unsigned char *a = base ? base + off : nullptr;
        off += (bytes + 255) / 256 * 256;
        return a;
    };
    unsigned char *self = take(sizeof(DevCase));
    unsigned char *p1 = take(sizeof(double) * (size_t)kMaxRed * d.red_stride);
    unsigned char *p2 = take(sizeof(double) * (size_t)kMaxRed * d.red_stride2);
    unsigned char *gt = take(sizeof(unsigned int) * (size_t)d.red_stride2);
    unsigned char *tk = take(sizeof(unsigned int) * 64);
    unsigned char *ks = take(sizeof(KState) * kNumKs);
    if (h) {
        h->self = reinterpret_cast<DevCase *>(self);
        h->partials = reinterpret_cast<double *>(p1);
        h->partials2 = reinterpret_cast<double *>(p2);
        h->gticket = reinterpret_cast<unsigned int *>(gt);
        h->ticket = reinterpret_cast<unsigned int *>(tk);
        h->ks = reinterpret_cast<KState *>(ks);
        h->ks_gather = nullptr;
    }
    return off;
}
}  // namespace

extern "C" fvm_status solve_pressure_static(fvm_case *c, const double *gamma, const double *rhs, double *p,
                                            const fvm_solver_ctl *ctl, void *stream, fvm_solve_info *out)
{
    if (!c || !gamma || !rhs || !p || !ctl) return fvm_fail(FVM_EINVAL, "solve_pressure_static: null argument");
    if (ctl->precond != FVM_PC_JACOBI)
        return fvm_fail(FVM_EINVAL, "solve_pressure_static: Jacobi preconditioning only");
    if (c->o.precision != FVM_FP64) return fvm_fail(FVM_EINVAL, "solve_pressure_static: FP64 cases only");
    if (ctl->max_iter < 1) return fvm_fail(FVM_EINVAL, "solve_pressure_static: max_iter must be >= 1");
    const size_t need = static_layout(c->d, nullptr, nullptr);
    if (need > kStaticScratchBytes)
        return fvm_fail(FVM_EINVAL, "solve_pressure_static: the case needs " + std::to_string(need) +
                                        " bytes of static scratch, more than its " +
                                        std::to_string(kStaticScratchBytes) + " (about 11M cells)");
    // the array used is the current device's: the case must live there
    int cur = -1;
    hipPointerAttribute_t pa{};
    if (hipGetDevice(&cur) != hipSuccess || hipPointerGetAttributes(&pa, c->d.p) != hipSuccess || pa.device != cur)
        return fvm_fail(FVM_EINVAL, "solve_pressure_static: the case's workspace is not on the current device");
    int herr = 0;
    unsigned char *base = static_cast<unsigned char *>(static_scratch(&herr));
    if (!base)
        return fvm_fail(FVM_EDEVICE, std::string("solve_pressure_static: static scratch address: ") +
                                         hipGetErrorString((hipError_t)herr));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    // descriptor whose reduction slots and Krylov states are in the scratch;
    // the vectors stay in the case's workspace
    DevCase h = c->d;
    static_layout(c->d, &h, base);
    const DevCase &d = c->d;
    HIPCHK(hipMemcpyAsync(h.self, &h, sizeof(DevCase), hipMemcpyHostToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    BatchSet bs;
    bs.n = 0;
    batch_add(bs, h.self, &h);
    launch_clear_reduction(bs, s);
    HIPCHK(hipMemcpyAsync(d.p_save, d.p, sizeof(double) * c->N, hipMemcpyDeviceToDevice, s));
    launch_gather_faces(bs, gamma, d.phiH, s);
    launch_p_system_from_gamma(bs, d.phiH, rhs, s);
    HIPCHK(hipMemcpyAsync(d.p, p, sizeof(double) * c->N, hipMemcpyDeviceToDevice, s));
    launch_set_ctl(bs, 3, 1, 2, ctl->tol, ctl->rel_tol, ctl->max_iter, s);
    launch_pcg_init(bs, 0, s);
    // direct launches in chunks, the stop flag read back after each chunk
    // (iterations past it return at once); no graph, no pinned buffer
    KState ks{};
    const long limit = (long)ctl->max_iter + 1;
    for (long issued = 0;;) {
        const long n = std::min<long>(8, limit - issued);
        for (long k = 0; k < n; ++k) launch_pcg_iter(bs, 0, (int)(k & 1), s);
        issued += n;
        HIPCHK(hipGetLastError());
        HIPCHK(hipMemcpyAsync(&ks, h.ks + 3, sizeof(KState), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (ks.done == 1) break;
        if (issued >= limit) return fvm_fail(FVM_EDEVICE, "solve_pressure_static: iteration limit passed without a stop flag");
    }
    if (ks.status >= 0) HIPCHK(hipMemcpyAsync(p, d.p, sizeof(double) * c->N, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipMemcpyAsync(d.p, d.p_save, sizeof(double) * c->N, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    if (out) to_info(ks, *out);
    if (ks.status < 0) return fvm_fail(ks.status, "solve_pressure_static: non-finite value or breakdown");
    return ks.status;
}

extern "C" fvm_status fvm_dic_apply(fvm_case *c, const double *gamma, const double *r, double *z, double *dstar,
                                    void *stream)
{
    if (!c || !gamma || !r || !z) return fvm_fail(FVM_EINVAL, "dic_apply: null argument");
    if (!c->d.dstar) return fvm_fail(FVM_EINVAL, "dic_apply: case was not created with the DIC preconditioner");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const Group g(c, s);
    const DevCase &d = c->d;
    launch_gather_faces(g.bs, gamma, d.phiH, s);
    launch_p_system_from_gamma(g.bs, d.phiH, r, s);
    HIPCHK(hipMemcpyAsync(d.r, r, sizeof(double) * c->N, hipMemcpyDeviceToDevice, s));
    launch_dic_reset(g.bs, s);
    launch_dic_precond(g.bs, 1, s);
    HIPCHK(hipMemcpyAsync(z, d.z, sizeof(double) * c->N, hipMemcpyDeviceToDevice, s));
    if (dstar) HIPCHK(hipMemcpyAsync(dstar, d.dstar, sizeof(double) * c->N, hipMemcpyDeviceToDevice, s));
    HIPCHK(hipStreamSynchronize(s));
    return FVM_OK;
}

extern "C" fvm_status fvm_case_operator(fvm_case *c, int32_t op, const double *d_in, double *d_out, void *stream)
{
    if (!c) return fvm_fail(FVM_EINVAL, "operator: null case");
    if (op < FVM_OP_GRAD || op > FVM_OP_HY_SETMAT) return fvm_fail(FVM_EINVAL, "operator: unknown op");
    if (op >= FVM_OP_HY_GRAD && c->d.hy_K <= 0)
        return fvm_fail(FVM_EINVAL, "operator: the case has no hybrid layout (create it with hybrid_K > 0)");
    if (c->o.precision != FVM_FP64) return fvm_fail(FVM_EINVAL, "operator: FP64 cases only");
    if (!d_in || (op != FVM_OP_HY_SETMAT && !d_out)) return fvm_fail(FVM_EINVAL, "operator: null array");
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const Group g(c, s);
    launch_operator(g.bs, op, d_in, d_out, s);
    HIPCHK(hipGetLastError());
    return FVM_OK;
}

extern "C" fvm_status piso_step_batch(fvm_case *const *cases, int32_t n, int32_t n_steps, void *stream,
                                      fvm_step_info *infos)
{
    if (!cases || n < 1 || n > kMaxBatch) return fvm_fail(FVM_EINVAL, "batch: need 1 <= n_cases <= 32");
    if (n_steps < 0) return fvm_fail(FVM_EINVAL, "piso: n_steps < 0");
    for (int i = 0; i < n; ++i) {
        const fvm_case *c = cases[i];
        if (!c) return fvm_fail(FVM_EINVAL, "batch: null case");
        if (!(c->o.dt > 0.0)) return fvm_fail(FVM_EINVAL, "piso: dt must be > 0");
        const fvm_case *a = cases[0];
        if (c->o.precision != a->o.precision || c->o.n_corr != a->o.n_corr ||
            c->o.n_non_orth_corr != a->o.n_non_orth_corr || c->o.p_ctl.precond != a->o.p_ctl.precond ||
            c->o.u_solver != a->o.u_solver)
            return fvm_fail(FVM_EINVAL, "batch: cases must share precision, correctors, preconditioner and momentum solver");
        if (n > 1 && c->o.p_ctl.precond == FVM_PC_AMG)
            return fvm_fail(FVM_EINVAL, "batch: AMG cases run one per call");
        for (int j = 0; j < i; ++j)
            if (cases[j] == c) return fvm_fail(FVM_EINVAL, "batch: a case appears twice");
    }
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    Poller *P = &cases[0]->poll;
    if (n > 1) {
        fvm_status st = t_batch_poll.init();
        if (st != FVM_OK) return st;
        P = &t_batch_poll;
    }
    Group g(cases, n, P, s);
    bool all_solo = true;
    for (int i = 0; i < n; ++i) all_solo = all_solo && cases[i]->solo();
    if (all_solo) return piso_solo(g, n_steps, infos);
    std::vector<int> idx(n);                 // group member -> caller's index
    for (int i = 0; i < n; ++i) idx[i] = i;
    std::vector<int32_t> acc(n, FVM_OK);
    std::vector<fvm_step_info> info;
    std::vector<fvm_step_info> last(n, fvm_step_info{});
    for (int32_t k = 0; k < n_steps; ++k) {
        Phase ph("piso step");
        launch_save(g.bs, 0, s);
        fvm_status st = piso_one(g, info);
        if (st != FVM_OK) return st;
        bool anyf = false;
        for (int j = 0; j < g.n(); ++j) {
            last[idx[j]] = info[j];
            worst(acc[idx[j]], info[j].status);
            anyf = anyf || info[j].status < 0;
        }
        if (anyf) {
            // failed cases are rolled back to the start of the step and leave
            // the batch; the others go on
            st = rollback_failed(g, info);
            if (st != FVM_OK) return st;
            std::vector<fvm_case *> keep;
            std::vector<int> kidx;
            for (int j = 0; j < g.n(); ++j)
                if (info[j].status >= 0) { keep.push_back(g.cs[j]); kidx.push_back(idx[j]); }
            if (keep.empty()) break;
            g = Group(keep.data(), (int)keep.size(), P, s);
            idx = kidx;
        }
    }
    // with an info record the call returns once all of its work is done,
    // so the fields may be read on any stream afterwards
    if (infos) HIPCHK(hipStreamSynchronize(s));
    // report in the caller's order
    int32_t all = FVM_OK;
    for (int i = 0; i < n; ++i) {
        if (infos) infos[i] = last[i];
        worst(all, acc[i]);
    }
    if (all < 0) return fvm_fail(all, "piso: a solve failed (non-finite value or breakdown); the case was rolled back");
    return all;
}
