// Host runtime behind the C ABI of include/sl.h: mesh object, validation,
// device buffers, time-step restriction, launch sequencing and statistics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <limits>
#include <shared_mutex>
#include <vector>

#include "sl_internal.h"

using namespace sl;

struct sl_mesh {
    int dim, kx, ky, n, nd, K, family, bc, form, precision;
    double x0, x1, y0, y1, dx, dy;
    hipStream_t stream;
    bool own_stream;
    BumpBlock* bump;  // buffers carved from this block (not freed here), or null: allocated
    Tables T;
    TabOff off;
    // device buffers
    double *phi, *phi2, *phihat, *rec, *eloc, *aN, *aM, *divN, *divM, *vface, *tab, *ghost, *stat_part;
    int32_t* flag_part;
    int32_t* vdeg_d;
    int nblocks;
    int nslice;  // statistics slices of nblocks blocks each: one per bucket of a mixed mesh, else 1
    int vdeg;
    // host state
    bool has_velocity;
    double amax[2];
    int ghost_rows;
    long ghost_step;
    double t;
    int64_t steps, steps_read;  // steps taken; value of steps at the last sl_read
    bool profiling;
    hipEvent_t ev[KER_COUNT][2];
    std::vector<hipEvent_t> pending[KER_COUNT];
    double ktime[KER_COUNT];
    int64_t kcount[KER_COUNT];
    // mixed-order meshes: elements grouped by order in buckets b (ascending
    // n); per-node arrays on the device are bucket after bucket
    bool mixed;
    int nbk;
    int bn[kMaxBuckets], bK[kMaxBuckets], bs[kMaxBuckets], bdeg[kMaxBuckets];
    size_t bOff[kMaxBuckets], aOff[kMaxBuckets], recOff[kMaxBuckets], tabOff[kMaxBuckets], elemOff[kMaxBuckets];
    std::vector<int32_t> orders;       // n_e per global element
    std::vector<size_t> uoff;          // caller layout offset of element e (n_e^2 values each)
    std::vector<size_t> doff;          // device (bucket) layout offset of element e
    int32_t *elems_d, *mix_d;
    int32_t* nbr_d;                    // [K][4 sides][3]: face partner table in bucket order (see MixFace)
    double *interp_d;
    size_t dofs;
    hipGraph_t graph;
    hipGraphExec_t gexec;
    bool graph_ok;
    double graph_dt;
    sl_step_opts graph_opts;
};

thread_local LaunchEvents sl::tl_timed_launch;
thread_local BumpBlock* sl::tl_bump = nullptr;

// per-kernel timing events (profiling) for kernel k.  A bracket around one
// launch (one_launch) hands its pair to that launch, which records the
// dispatch's own start and end (launch_timed); a bracket around several
// launches records the pair on the stream before and after them.
void ev_begin(sl_mesh* m, int k, bool one_launch)
{
    if (!m->profiling) return;
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    if (one_launch)
        tl_timed_launch = LaunchEvents{a, b};
    else
        (void)hipEventRecord(a, m->stream);
    m->pending[k].push_back(a);
    m->pending[k].push_back(b);
}

void ev_end(sl_mesh* m, int k, bool one_launch)
{
    if (!m->profiling) return;
    if (!one_launch) {
        (void)hipEventRecord(m->pending[k].back(), m->stream);
    } else if (tl_timed_launch.start) {
        // no launch took the pair: it carries no time
        tl_timed_launch = LaunchEvents{};
        for (int i = 0; i < 2; ++i) {
            (void)hipEventDestroy(m->pending[k].back());
            m->pending[k].pop_back();
        }
    }
}

namespace {

// number of velocity series terms the 1D advect kernel evaluates (mirrors
// the choice in launch_adv_n: 4, 8 or all n)
int vel_terms_used(const sl_mesh* m)
{
    const int need = m->vdeg + 1, n = m->n;
    if (m->dim == 2) return need;  // 2D evaluates exactly vdeg + 1 terms per direction
    if (n > 4 && need <= 4) return 4;
    if (n > 8 && need <= 8) return 8;
    return n;
}

template <typename T>
void dfree(const sl_mesh* m, T*& p)
{
    if (p && !m->bump) (void)hipFree(p);
    p = nullptr;
}

void release(sl_mesh* m)
{
    dfree(m, m->phi); dfree(m, m->phi2); dfree(m, m->phihat); dfree(m, m->rec); dfree(m, m->eloc); dfree(m, m->aN);
    dfree(m, m->aM); dfree(m, m->divN); dfree(m, m->divM); dfree(m, m->vface); dfree(m, m->tab); dfree(m, m->ghost);
    dfree(m, m->stat_part); dfree(m, m->flag_part); dfree(m, m->vdeg_d);
    dfree(m, m->elems_d); dfree(m, m->mix_d); dfree(m, m->interp_d); dfree(m, m->nbr_d);
    if (m->gexec) (void)hipGraphExecDestroy(m->gexec);
    if (m->graph) (void)hipGraphDestroy(m->graph);
    m->gexec = nullptr;
    m->graph = nullptr;
    for (int k = 0; k < KER_COUNT; ++k)
        for (hipEvent_t e : m->pending[k]) (void)hipEventDestroy(e);
    if (m->own_stream && m->stream) (void)hipStreamDestroy(m->stream);
}

bool all_finite(const double* p, size_t n)
{
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(p[i])) return false;
    return true;
}

template <typename T>
bool dalloc(const sl_mesh* m, T** p, size_t count)
{
    if (count == 0) count = 1;
    if (BumpBlock* b = m->bump) {
        const size_t at = (b->used + 255) / 256 * 256, bytes = count * sizeof(T);
        if (at > b->size || bytes > b->size - at) return false;
        *p = reinterpret_cast<T*>(b->base + at);
        b->used = at + bytes;
        return true;
    }
    return hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T)) == hipSuccess;
}

// element counts of a mesh's device buffers (the single place that sizes them)
struct BufSizes {
    size_t nf, nrec, nvf, ntab, nstat, nflag;
    size_t ncoef;  // velocity coefficients: dim * nf, and in 1D the [K][4] copies of aM and divM after them
    int nblocks;
};
BufSizes buffer_sizes(int dim, int kx, int ky, int n)
{
    BufSizes z;
    const size_t K = (size_t)kx * ky;
    z.nf = K * (dim == 1 ? n : n * n);
    z.nblocks = dim == 1 ? blocks1d(n, (int)K) : blocks2d(n, (int)K);
    // 2D: traces (4n), stage sums (8n), targets (2), backtraced face values (4n)
    z.nrec = dim == 1 ? K * kRec1 : K * (16 * n + 3);
    z.nvf = dim == 1 ? K + 1 : K * 4 * n;
    z.ntab = (size_t)tab_offsets(dim, n).total;
    z.nstat = (size_t)z.nblocks * kStatSlots;
    z.nflag = (size_t)2 * z.nblocks;
    z.ncoef = z.nf * dim + (dim == 1 ? 8 * K : 0);
    return z;
}

// 2D Gram constants are not needed; 1D rows l(0), l(1), W

}  // namespace

namespace sl {

TabOff tab_offsets(int dim, int n)
{
    TabOff o;
    o.xi = 0;
    o.w = n;
    o.l0 = 2 * n;
    o.l1 = 3 * n;
    o.tinv = 4 * n;
    o.dmat = 4 * n + n * n;
    o.lam = 4 * n + 2 * n * n;
    o.cbp = o.lam + n;
    o.softs = o.cbp + (dim == 2 ? 16 * n * n : 0);
    o.zmh = o.softs + (dim == 2 ? 16 * n * n : 0);
    o.zms = o.zmh + (dim == 2 ? n * n : 0);
    o.total = o.zms + (dim == 2 ? n * n : 0);
    return o;
}

bool rk_tableau(int order, RKTab* T)
{
    std::memset(T, 0, sizeof(*T));
    switch (order) {
    case 1: T->s = 1; T->b[0] = 1; break;
    case 2: T->s = 2; T->a[1][0] = 1; T->b[0] = 0.5; T->b[1] = 0.5; T->c[1] = 1; break;
    case 3:
        T->s = 3; T->a[1][0] = 0.5; T->a[2][0] = -1; T->a[2][1] = 2;
        T->b[0] = 1.0 / 6; T->b[1] = 2.0 / 3; T->b[2] = 1.0 / 6; T->c[1] = 0.5; T->c[2] = 1;
        break;
    case 4:
        T->s = 4; T->a[1][0] = 0.5; T->a[2][1] = 0.5; T->a[3][2] = 1;
        T->b[0] = 1.0 / 6; T->b[1] = 1.0 / 3; T->b[2] = 1.0 / 3; T->b[3] = 1.0 / 6;
        T->c[1] = 0.5; T->c[2] = 0.5; T->c[3] = 1;
        break;
    default: return false;
    }
    T->nq = 0;
    for (int s = 0; s < T->s; ++s) {
        int f = -1;
        for (int q = 0; q < T->nq; ++q)
            if (T->cu[q] == T->c[s]) f = q;
        if (f < 0) { T->cu[T->nq] = T->c[s]; T->bu[T->nq] = T->b[s]; ++T->nq; }
        else T->bu[f] += T->b[s];
    }
    return true;
}

namespace {
std::shared_mutex g_dev_mu;
thread_local int tl_hold = 0;  // depth of this thread's ApiHold
}  // namespace

ApiHold::ApiHold()
{
    if (tl_hold++ == 0) g_dev_mu.lock_shared();
}
ApiHold::~ApiHold()
{
    if (--tl_hold == 0) g_dev_mu.unlock_shared();
}
CaptureHold::CaptureHold() : saved(tl_hold)
{
    if (saved) g_dev_mu.unlock_shared();
    tl_hold = 0;
    g_dev_mu.lock();
}
CaptureHold::~CaptureHold()
{
    g_dev_mu.unlock();
    tl_hold = saved;
    if (saved) g_dev_mu.lock_shared();
}

bool step_opts_valid(const sl_step_opts& opt)
{
    return opt.rk >= 1 && opt.rk <= 4 && !(opt.constraints & ~7) &&
           (opt.mode == SL_MODE_HARD || opt.mode == SL_MODE_SOFT) && opt.energy_maxit >= 0 &&
           opt.energy_tol >= 0 && opt.refine_steps >= 0 &&
           (opt.iface == SL_IFACE_INTERP || opt.iface == SL_IFACE_BACKTRACK);
}

bool step1d_setup(const Tables& T, int n, double dx, int periodic, int cons, const sl_step_opts& opt, double amax,
                  Step1DArgs* A)
{
    rk_tableau(opt.rk, &A->rk);
    A->periodic = periodic;
    A->cons = cons;
    A->cmask = opt.constraints; A->mode = opt.mode; A->emaxit = opt.energy_maxit; A->etol = opt.energy_tol;
    A->iface = opt.iface;
    A->targets = (opt.constraints & (SL_C_MASS | SL_C_ENERGY)) != 0;
    A->vol = A->targets;
    A->dx = dx; A->invdx = 1.0 / dx;
    A->vzero = 1e-12 * amax;
    // Gram entries of the rows l(0), l(1) (boundary) and W (mass)
    double g00 = 0, g01 = 0, g11 = 0, g02 = 0, g12 = 0, g22 = 0;
    A->sumW = 0.0;
    for (int j = 0; j < n; ++j) {
        const double W = dx * T.w[j];
        g00 += T.l0[j] * T.l0[j];
        g01 += T.l0[j] * T.l1[j];
        g11 += T.l1[j] * T.l1[j];
        g02 += T.l0[j] * W;
        g12 += T.l1[j] * W;
        g22 += W * W;
        A->sumW += W;
    }
    A->g00 = g00; A->g01 = g01; A->g11 = g11; A->g02 = g02; A->g12 = g12; A->g22 = g22;
    // the block of the constrained system that does not depend on the
    // element: rows l(0), l(1) (boundary) and W (mass); an inactive row is an
    // identity row, SOFT adds I
    const bool bnd = (opt.constraints & SL_C_BOUNDARY) != 0, mass = (opt.constraints & SL_C_MASS) != 0;
    const bool ac[3] = {bnd, bnd, mass};
    double G3[9] = {bnd ? g00 : 0.0, bnd ? g01 : 0.0, (bnd && mass) ? g02 : 0.0,
                    bnd ? g01 : 0.0, bnd ? g11 : 0.0, (bnd && mass) ? g12 : 0.0,
                    (bnd && mass) ? g02 : 0.0, (bnd && mass) ? g12 : 0.0, mass ? g22 : 0.0};
    for (int a = 0; a < 3; ++a) {
        if (opt.mode == SL_MODE_HARD && !ac[a]) G3[a * 3 + a] = 1.0;
        if (opt.mode == SL_MODE_SOFT) G3[a * 3 + a] += 1.0;
    }
    return invert(3, G3, A->g3i);
}

}  // namespace sl


// ===========================================================================
// mixed-order meshes
// ===========================================================================
namespace {

// Lagrange basis of nodes xf[0..nf) at x, product form (exact at the nodes)
double lag_at(const double* xf, int nf, int j, double x)
{
    double v = 1.0;
    for (int i = 0; i < nf; ++i)
        if (i != j) v *= (x - xf[i]) / (xf[j] - xf[i]);
    return v;
}

struct MixedPlan {
    int nbk = 0;
    int bn[kMaxBuckets] = {}, bK[kMaxBuckets] = {};
    size_t dofs = 0, nrec = 0, ntab = 0, ninterp = 0;
    int nblocks = 1;
};

// buckets and buffer sizes of a mixed-order descriptor (validated)
bool mixed_plan(const sl_mesh_desc* d, MixedPlan* P)
{
    if (d->dim != 2 || d->bc != SL_BC_PERIODIC || d->kx < 1 || d->ky < 1) return false;
    if ((int64_t)d->kx * d->ky > (1 << 26)) return false;
    const int K = d->kx * d->ky;
    int count[kMax2D + 1] = {};
    for (int e = 0; e < K; ++e) {
        const int n = d->orders[e] + 1;
        if (d->orders[e] < 1 || n > kMax2D) return false;
        ++count[n];
    }
    for (int n = 2; n <= kMax2D; ++n)
        if (count[n]) {
            const int b = P->nbk++;
            P->bn[b] = n;
            P->bK[b] = count[n];
            P->dofs += (size_t)count[n] * n * n;
            P->nrec += (size_t)count[n] * 4 * n;
            P->ntab += (size_t)tab_offsets(2, n).total;
            P->nblocks = std::max(P->nblocks, count[n]);
        }
    for (int a = 0; a < P->nbk; ++a)
        for (int b = 0; b < P->nbk; ++b)
            if (a != b) P->ninterp += (size_t)P->bn[a] * P->bn[b];
    return true;
}

size_t mixed_bytes(const sl_mesh_desc* d, const MixedPlan& P)
{
    const size_t K = (size_t)d->kx * d->ky;
    const size_t dbl = 3 * P.dofs + 2 * 2 * P.dofs + 2 * P.dofs + 2 * P.nrec + P.ntab + P.ninterp +
                       (size_t)P.nbk * P.nblocks * kStatSlots;
    const size_t ints =
        2 * (size_t)P.nbk * P.nblocks + 1 + K + (size_t)MixMeta::size((int)K) + K * MixFace::kPer;
    return dbl * sizeof(double) + ints * sizeof(int32_t);
}

// per-bucket arguments of one launch; phi pointers are set per step
Step2DArgs bucket_args(const sl_mesh* m, int b, double dt, const sl_step_opts& opt)
{
    Step2DArgs B;
    std::memset(&B, 0, sizeof(B));
    rk_tableau(opt.rk, &B.rk);
    const int n = m->bn[b];
    B.phihat = m->phihat + m->bOff[b];
    B.rec = m->rec + m->recOff[b];
    B.aN = m->aN + m->aOff[b];
    B.aM = m->aM + m->aOff[b];
    B.divN = m->divN + m->bOff[b];
    B.divM = m->divM + m->bOff[b];
    B.vface = m->vface + m->recOff[b];
    B.tab = m->tab + m->tabOff[b];
    B.gnow = B.gnext = m->vface;
    // each bucket keeps its block statistics in a slice of its own
    B.flag_part = m->flag_part + (size_t)b * 2 * m->nblocks;
    B.stat_part = m->stat_part + (size_t)b * m->nblocks * kStatSlots;
    B.nblk = m->nblocks;
    B.vdeg = m->bdeg[b];
    B.rstride = 4 * n;
    B.kx = m->kx;
    B.ky = m->ky;
    B.K = m->bK[b];
    B.periodic = 3;
    B.cons = m->form == SL_FORM_CONSERVATIVE;
    B.cmask = opt.constraints;
    B.mode = opt.mode;
    B.refine = 60;
    B.precision = m->precision;
    B.dx = m->dx;
    B.dy = m->dy;
    B.invdx = 1.0 / m->dx;
    B.invdy = 1.0 / m->dy;
    B.dt = dt;
    B.vzero = 1e-12 * std::max(m->amax[0], m->amax[1]);
    B.bs = m->bs[b] > 0 ? m->bs[b] : 0;
    B.elems = m->elems_d + m->elemOff[b];
    B.mix = m->mix_d;
    B.nbr = m->nbr_d + m->elemOff[b] * MixFace::kPer;
    B.rec_all = m->rec;
    B.interp = m->interp_d;
    B.bucket = b;
    return B;
}

// one step of every bucket: all advects (each writes its records), then all
// constraints (each reads the neighbours' records); with profiling every
// launch is bracketed by events
int mixed_launch_step(sl_mesh* m, std::vector<Step2DArgs>& B, double* src, double* dst)
{
    for (int b = 0; b < m->nbk; ++b) {
        B[b].phi = src + m->bOff[b];
        B[b].phi_out = dst + m->bOff[b];
        ev_begin(m, KER_MIX_ADV + b, true);
        if (launch_advect2d(m->bn[b], B[b], m->stream)) return 1;
        ev_end(m, KER_MIX_ADV + b, true);
    }
    for (int b = 0; b < m->nbk; ++b) {
        ev_begin(m, KER_MIX_CON + b, true);
        if (launch_constrain2d_mixed(m->bn[b], B[b], m->stream)) return 1;
        ev_end(m, KER_MIX_CON + b, true);
    }
    return 0;
}

// pick, per bucket, the fastest block shape of the advect kernel on the
// mesh's own data (three timed launches per shape); the statistics the
// trial launches accumulate are cleared afterwards
sl_status mixed_autotune(sl_mesh* m, double dt, const sl_step_opts& opt)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) || hipEventCreate(&e1)) return SL_E_DEVICE;
    sl_status rc = SL_OK;
    for (int b = 0; b < m->nbk && rc == SL_OK; ++b) {
        Step2DArgs B = bucket_args(m, b, dt, opt);
        B.phi = m->phi + m->bOff[b];
        B.phi_out = m->phi2 + m->bOff[b];
        float best = 1e30f;
        int pick = 0;
        for (int sh = 0; sh < advect2d_shapes(m->bn[b]) && rc == SL_OK; ++sh) {
            if (advect2d_elems(m->bn[b], sh) < 1) continue;
            B.bs = sh;
            if (launch_advect2d(m->bn[b], B, m->stream)) { rc = SL_E_DEVICE; break; }
            (void)hipEventRecord(e0, m->stream);
            for (int r = 0; r < 3; ++r)
                if (launch_advect2d(m->bn[b], B, m->stream)) rc = SL_E_DEVICE;
            (void)hipEventRecord(e1, m->stream);
            float ms = 0.0f;
            if (hipEventSynchronize(e1) || hipEventElapsedTime(&ms, e0, e1)) rc = SL_E_DEVICE;
            if (rc == SL_OK && ms < best) { best = ms; pick = sh; }
        }
        m->bs[b] = pick;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != SL_OK) return rc;
    if (hipMemsetAsync(m->stat_part, 0, (size_t)m->nslice * m->nblocks * kStatSlots * sizeof(double), m->stream) ||
        hipMemsetAsync(m->flag_part, 0, (size_t)m->nslice * 2 * m->nblocks * sizeof(int32_t), m->stream))
        return SL_E_DEVICE;
    return SL_OK;
}

}  // namespace

extern "C" {

const char* sl_status_string(sl_status s)
{
    switch (s) {
    case SL_OK: return "ok";
    case SL_E_INVALID: return "invalid argument";
    case SL_E_NOMEM: return "out of device memory";
    case SL_E_DEVICE: return "device error";
    case SL_E_STATE: return "invalid state";
    case SL_E_CFL: return "time step lets particles leave their element";
    case SL_E_NONFINITE: return "non-finite value";
    case SL_E_SINGULAR: return "singular system";
    case SL_E_NOCONV: return "energy iteration did not converge";
    default: return "unknown status";
    }
}

sl_status sl_node_coords(int32_t nodes, int32_t n, double* xi, double* w)
{
    if (!xi || !w || n < 1 || n > kMaxTableN) return SL_E_INVALID;
    return node_rule(nodes, n, xi, w) ? SL_OK : SL_E_INVALID;
}

// mixed-order mesh: buckets, tables, interpolation matrices, meta data and
// the initial field in bucket layout (validated by mixed_plan)
static sl_status create_mixed(const sl_mesh_desc* d, sl_mesh** out)
{
    MixedPlan P;
    if (!mixed_plan(d, &P)) return SL_E_INVALID;
    if (d->nodes != SL_NODES_GL && d->nodes != SL_NODES_CG) return SL_E_INVALID;
    if (d->form != SL_FORM_ADVECTIVE && d->form != SL_FORM_CONSERVATIVE) return SL_E_INVALID;
    if (d->precision != SL_PREC_FP64 && d->precision != SL_PREC_FP32_REFINED && d->precision != SL_PREC_BF16_REFINED)
        return SL_E_INVALID;
    // above 16 nodes per direction the 2D kernels are FP64 only
    for (int b = 0; b < P.nbk; ++b)
        if (P.bn[b] > kMax2DFull && d->precision != SL_PREC_FP64) return SL_E_INVALID;
    if (!(d->x1 > d->x0) || !(d->y1 > d->y0) || !std::isfinite(d->x0) || !std::isfinite(d->x1) ||
        !std::isfinite(d->y0) || !std::isfinite(d->y1))
        return SL_E_INVALID;
    const int K = d->kx * d->ky;
    if (!all_finite(d->u0, P.dofs)) return SL_E_NONFINITE;
    sl_mesh* m = new (std::nothrow) sl_mesh();
    if (!m) return SL_E_NOMEM;
    m->bump = tl_bump;
    m->mixed = true;
    m->dim = 2; m->kx = d->kx; m->ky = d->ky; m->K = K;
    m->family = d->nodes; m->bc = d->bc; m->form = d->form; m->precision = d->precision;
    m->x0 = d->x0; m->x1 = d->x1; m->y0 = d->y0; m->y1 = d->y1;
    m->dx = (d->x1 - d->x0) / d->kx;
    m->dy = (d->y1 - d->y0) / d->ky;
    m->nbk = P.nbk;
    m->n = P.bn[P.nbk - 1];  // largest order: its edge gap is the smallest
    m->nd = m->n * m->n;
    m->dofs = P.dofs;
    if (!build_tables(m->family, m->n, &m->T)) { delete m; return SL_E_INVALID; }
    m->off = tab_offsets(2, m->n);
    // bucket offsets
    size_t bo = 0, ro = 0, to = 0, eo = 0;
    for (int b = 0; b < P.nbk; ++b) {
        const int n = P.bn[b];
        m->bn[b] = n;
        m->bK[b] = P.bK[b];
        m->bs[b] = -1;
        m->bOff[b] = bo;
        m->aOff[b] = 2 * bo;
        m->recOff[b] = ro;
        m->tabOff[b] = to;
        m->elemOff[b] = eo;
        bo += (size_t)P.bK[b] * n * n;
        ro += (size_t)P.bK[b] * 4 * n;
        to += (size_t)tab_offsets(2, n).total;
        eo += (size_t)P.bK[b];
    }
    // the device meta data and face table hold these offsets as int32
    if (2 * bo > (size_t)std::numeric_limits<int32_t>::max() || ro > (size_t)std::numeric_limits<int32_t>::max()) {
        delete m;
        return SL_E_INVALID;
    }
    // element placement: caller layout (element order) and bucket layout
    int bucket_of[kMax2D + 1];
    for (int b = 0; b < P.nbk; ++b) bucket_of[P.bn[b]] = b;
    std::vector<int32_t> meta((size_t)MixMeta::size(K), 0), elems((size_t)K);
    m->orders.resize(K);
    m->uoff.resize(K);
    m->doff.resize(K);
    int fill[kMaxBuckets] = {};
    size_t uo = 0;
    for (int e = 0; e < K; ++e) {
        const int n = d->orders[e] + 1, b = bucket_of[n], idx = fill[b]++;
        m->orders[e] = n;
        m->uoff[e] = uo;
        uo += (size_t)n * n;
        m->doff[e] = m->bOff[b] + (size_t)idx * n * n;
        meta[e] = b;
        meta[(size_t)K + e] = idx;
        elems[m->elemOff[b] + idx] = e;
    }
    int32_t* mm = meta.data() + 2 * (size_t)K;
    for (int b = 0; b < P.nbk; ++b) {
        mm[MixMeta::kN + b] = P.bn[b];
        mm[MixMeta::kRec + b] = (int32_t)m->recOff[b];
        mm[MixMeta::kVel + b] = (int32_t)m->aOff[b];
        mm[MixMeta::kTab + b] = (int32_t)m->tabOff[b];
        mm[MixMeta::kK + b] = P.bK[b];
    }
    // tables per bucket, interpolation matrices between bucket orders
    std::vector<double> tab(P.ntab, 0.0), interp(std::max<size_t>(P.ninterp, 1), 0.0);
    std::vector<Tables> T(P.nbk);
    bool ok = true;
    for (int b = 0; b < P.nbk && ok; ++b) {
        const int n = P.bn[b];
        ok = build_tables(m->family, n, &T[b]);
        if (!ok) break;
        const TabOff o = tab_offsets(2, n);
        double* tb = tab.data() + m->tabOff[b];
        for (int j = 0; j < n; ++j) {
            tb[o.xi + j] = T[b].xi[j];
            tb[o.w + j] = T[b].w[j];
            tb[o.l0 + j] = T[b].l0[j];
            tb[o.l1 + j] = T[b].l1[j];
            tb[o.lam + j] = T[b].lam[j];
            for (int k = 0; k < n; ++k) {
                tb[o.tinv + j * n + k] = T[b].Tinv[j * n + k];
                tb[o.dmat + j * n + k] = T[b].D[j * n + k];
            }
        }
        ok = build_boundary_tables(T[b], tb + o.cbp, tb + o.softs, tb + o.zmh, tb + o.zms);
    }
    size_t io = 0;
    for (int a = 0; a < P.nbk && ok; ++a)
        for (int b = 0; b < P.nbk; ++b) {
            if (a == b) continue;
            mm[MixMeta::kInterp + kMaxBuckets * a + b] = (int32_t)io;
            for (int k = 0; k < P.bn[a]; ++k)
                for (int j = 0; j < P.bn[b]; ++j)
                    interp[io + (size_t)k * P.bn[b] + j] = lag_at(T[b].xi, P.bn[b], j, T[a].xi[k]);
            io += (size_t)P.bn[a] * P.bn[b];
        }
    if (!ok) { delete m; return SL_E_INVALID; }
    // face partner table, in bucket order: for each side of each element the
    // neighbour's matching trace row in the records of all buckets, its
    // order, and the interpolation matrix from its order (-1: the same)
    std::vector<int32_t> nbr((size_t)K * MixFace::kPer);
    for (int e = 0; e < K; ++e) {
        const int b = meta[e], pos = (int)m->elemOff[b] + meta[(size_t)K + e];
        const int ex = e % d->kx, ey = e / d->kx;
        for (int side = 0; side < 4; ++side) {
            int nbe;
            switch (side) {
            case 0: nbe = ey * d->kx + (ex + d->kx - 1) % d->kx; break;
            case 1: nbe = ey * d->kx + (ex + 1) % d->kx; break;
            case 2: nbe = ((ey + d->ky - 1) % d->ky) * d->kx + ex; break;
            default: nbe = ((ey + 1) % d->ky) * d->kx + ex; break;
            }
            const int b2 = meta[nbe], j2 = meta[(size_t)K + nbe], n2 = P.bn[b2];
            int32_t* f = &nbr[(size_t)pos * MixFace::kPer + side * MixFace::kField];
            f[MixFace::kRecOff] = (int32_t)(m->recOff[b2] + (size_t)j2 * 4 * n2 + (size_t)(side ^ 1) * n2);
            f[MixFace::kOrder] = n2;
            f[MixFace::kInterpOff] = b2 == b ? -1 : mm[MixMeta::kInterp + kMaxBuckets * b + b2];
        }
    }
    if (d->stream) { m->stream = (hipStream_t)d->stream; m->own_stream = false; }
    else {
        if (hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking) != hipSuccess) { delete m; return SL_E_DEVICE; }
        m->own_stream = true;
    }
    m->nblocks = P.nblocks;
    m->nslice = P.nbk;
    ok = dalloc(m, &m->phi, P.dofs) && dalloc(m, &m->phi2, P.dofs) && dalloc(m, &m->phihat, P.dofs) &&
         dalloc(m, &m->rec, P.nrec) && dalloc(m, &m->aN, 2 * P.dofs) && dalloc(m, &m->aM, 2 * P.dofs) &&
         dalloc(m, &m->divN, P.dofs) && dalloc(m, &m->divM, P.dofs) && dalloc(m, &m->vface, P.nrec) &&
         dalloc(m, &m->tab, P.ntab) && dalloc(m, &m->stat_part, (size_t)m->nslice * m->nblocks * kStatSlots) &&
         dalloc(m, &m->flag_part, (size_t)m->nslice * 2 * m->nblocks) && dalloc(m, &m->vdeg_d, 1) && dalloc(m, &m->elems_d, (size_t)K) &&
         dalloc(m, &m->mix_d, meta.size()) && dalloc(m, &m->interp_d, interp.size()) && dalloc(m, &m->nbr_d, nbr.size());
    if (!ok) { release(m); delete m; return SL_E_NOMEM; }
    std::vector<double> u((size_t)P.dofs);
    for (int e = 0; e < K; ++e)
        std::memcpy(&u[m->doff[e]], d->u0 + m->uoff[e], sizeof(double) * m->orders[e] * m->orders[e]);
    hipError_t r[9] = {
        hipMemcpyAsync(m->nbr_d, nbr.data(), nbr.size() * sizeof(int32_t), hipMemcpyHostToDevice, m->stream),
        hipMemcpyAsync(m->tab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, m->stream),
        hipMemcpyAsync(m->phi, u.data(), u.size() * sizeof(double), hipMemcpyHostToDevice, m->stream),
        hipMemcpyAsync(m->elems_d, elems.data(), elems.size() * sizeof(int32_t), hipMemcpyHostToDevice, m->stream),
        hipMemcpyAsync(m->mix_d, meta.data(), meta.size() * sizeof(int32_t), hipMemcpyHostToDevice, m->stream),
        hipMemcpyAsync(m->interp_d, interp.data(), interp.size() * sizeof(double), hipMemcpyHostToDevice, m->stream),
        hipMemsetAsync(m->stat_part, 0, (size_t)m->nslice * m->nblocks * kStatSlots * sizeof(double), m->stream),
        hipMemsetAsync(m->flag_part, 0, (size_t)m->nslice * 2 * m->nblocks * sizeof(int32_t), m->stream),
        hipStreamSynchronize(m->stream)};
    for (hipError_t x : r)
        if (x != hipSuccess) { release(m); delete m; return SL_E_DEVICE; }
    *out = m;
    return SL_OK;
}

// velocity of a mixed-order mesh: to bucket layout, then per bucket the
// series coefficients and effective degree, then the face speeds
static sl_status set_velocity_mixed(sl_mesh* m, const double* a, const double* div_a)
{
    const size_t nf = m->dofs;
    if (!all_finite(a, 2 * nf)) return SL_E_NONFINITE;
    if (div_a && !all_finite(div_a, nf)) return SL_E_NONFINITE;
    double am[2] = {0.0, 0.0};
    for (int c = 0; c < 2; ++c)
        for (size_t i = 0; i < nf; ++i) am[c] = std::max(am[c], std::fabs(a[c * nf + i]));
    // steps already queued on the mesh's stream read the velocity arrays:
    // let them finish before the copies below overwrite them
    if (hipStreamSynchronize(m->stream)) return SL_E_DEVICE;
    std::vector<double> da(2 * nf), dd(div_a ? nf : 0);
    for (int e = 0; e < m->K; ++e) {
        const int n = m->orders[e], nd = n * n;
        int b = 0;
        while (m->bn[b] != n) ++b;
        const size_t idx = (m->doff[e] - m->bOff[b]) / nd;
        std::memcpy(&da[m->aOff[b] + idx * nd], a + m->uoff[e], sizeof(double) * nd);
        std::memcpy(&da[m->aOff[b] + ((size_t)m->bK[b] + idx) * nd], a + nf + m->uoff[e], sizeof(double) * nd);
        if (div_a) std::memcpy(&dd[m->doff[e]], div_a + m->uoff[e], sizeof(double) * nd);
    }
    if (hipMemcpy(m->aN, da.data(), da.size() * sizeof(double), hipMemcpyHostToDevice)) return SL_E_DEVICE;
    if (div_a && hipMemcpy(m->divN, dd.data(), dd.size() * sizeof(double), hipMemcpyHostToDevice)) return SL_E_DEVICE;
    const int cons = m->form == SL_FORM_CONSERVATIVE;
    int vmax = 0;
    for (int b = 0; b < m->nbk; ++b) {
        int32_t deg = m->bn[b] - 1;
        if (hipMemsetAsync(m->vdeg_d, 0, sizeof(int32_t), m->stream) ||
            launch_prep2d(m->bn[b], m->bK[b], div_a != nullptr, cons, m->aN + m->aOff[b], m->aM + m->aOff[b],
                          m->divN + m->bOff[b], m->divM + m->bOff[b], m->tab + m->tabOff[b], m->dx, m->dy,
                          std::max(am[0], am[1]), m->vdeg_d, m->stream) ||
            hipMemcpyAsync(&deg, m->vdeg_d, sizeof(int32_t), hipMemcpyDeviceToHost, m->stream) ||
            hipStreamSynchronize(m->stream))
            return SL_E_DEVICE;
        m->bdeg[b] = deg;
        vmax = std::max(vmax, deg);
    }
    const double vzero = 1e-12 * std::max(am[0], am[1]);
    for (int b = 0; b < m->nbk; ++b)
        if (launch_facevel2d_mixed(m->bn[b], m->bK[b], b, m->kx, m->ky, m->elems_d + m->elemOff[b], m->mix_d, m->aN,
                                   m->tab, m->interp_d, vzero, m->vface + m->recOff[b], m->stream))
            return SL_E_DEVICE;
    if (hipStreamSynchronize(m->stream)) return SL_E_DEVICE;
    m->vdeg = vmax;
    m->amax[0] = am[0];
    m->amax[1] = am[1];
    m->has_velocity = true;
    m->graph_ok = false;  // the captured launches carry the degrees
    return SL_OK;
}

// steps of a mixed-order mesh (validated by sl_step): autotune once, then
// replay a captured two-step graph; an odd last step runs eagerly
static sl_status step_mixed(sl_mesh* m, double dt, int32_t nsteps, const sl_step_opts& opt)
{
    if (opt.constraints & (SL_C_MASS | SL_C_ENERGY)) return SL_E_INVALID;
    bool tuned = true;
    for (int b = 0; b < m->nbk; ++b) tuned = tuned && m->bs[b] >= 0;
    if (!tuned) {
        const sl_status rc = mixed_autotune(m, dt, opt);
        if (rc != SL_OK) return rc;
        m->graph_ok = false;
    }
    std::vector<Step2DArgs> B(m->nbk);
    for (int b = 0; b < m->nbk; ++b) B[b] = bucket_args(m, b, dt, opt);
    int32_t done = 0;
    if (!m->profiling && nsteps >= 2) {
        const bool same = m->graph_ok && m->graph_dt == dt && !std::memcmp(&m->graph_opts, &opt, sizeof(opt));
        if (!same) {
            if (m->gexec) (void)hipGraphExecDestroy(m->gexec);
            if (m->graph) (void)hipGraphDestroy(m->graph);
            m->gexec = nullptr;
            m->graph = nullptr;
            m->graph_ok = false;
            // the capture holds out this library's allocating and
            // synchronising calls in other threads
            const CaptureHold excl;
            if (hipStreamBeginCapture(m->stream, hipStreamCaptureModeThreadLocal)) return SL_E_DEVICE;
            const int bad = mixed_launch_step(m, B, m->phi, m->phi2) | mixed_launch_step(m, B, m->phi2, m->phi);
            hipGraph_t g = nullptr;
            const hipError_t ec = hipStreamEndCapture(m->stream, &g);
            if (bad || ec != hipSuccess || !g) {
                if (g) (void)hipGraphDestroy(g);
                return SL_E_DEVICE;
            }
            m->graph = g;
            if (hipGraphInstantiate(&m->gexec, m->graph, nullptr, nullptr, 0)) return SL_E_DEVICE;
            m->graph_ok = true;
            m->graph_dt = dt;
            m->graph_opts = opt;
        }
        // the graph reads the field from m->phi and leaves it there
        for (; done + 2 <= nsteps; done += 2)
            if (hipGraphLaunch(m->gexec, m->stream)) return SL_E_DEVICE;
    }
    for (; done < nsteps; ++done) {
        ev_begin(m, KER_ADV2D, false);
        if (mixed_launch_step(m, B, m->phi, m->phi2)) return SL_E_DEVICE;
        ev_end(m, KER_ADV2D, false);
        // the graph captured m->phi as its input: bring the field back there
        if (hipMemcpyAsync(m->phi, m->phi2, m->dofs * sizeof(double), hipMemcpyDeviceToDevice, m->stream))
            return SL_E_DEVICE;
    }
    m->t += dt * nsteps;
    m->steps += nsteps;
    return SL_OK;
}

sl_status sl_create_mesh(const sl_mesh_desc* d, sl_mesh** out)
{
    const ApiHold hold;
    if (!out) return SL_E_INVALID;
    *out = nullptr;
    if (!d || !d->u0) return SL_E_INVALID;
    if (d->orders) return create_mixed(d, out);
    if (d->dim != 1 && d->dim != 2) return SL_E_INVALID;
    const int n = d->order + 1;
    if (d->order < 1 || n > (d->dim == 1 ? kMax1D : kMax2D)) return SL_E_INVALID;
    if (d->kx < 1 || d->ky < 1 || (d->dim == 1 && d->ky != 1)) return SL_E_INVALID;
    if ((int64_t)d->kx * d->ky > (1 << 26)) return SL_E_INVALID;
    if (d->nodes != SL_NODES_GL && d->nodes != SL_NODES_CG) return SL_E_INVALID;
    if (d->bc != SL_BC_PERIODIC && d->bc != SL_BC_GHOST &&
        !(d->dim == 2 && (d->bc == SL_BC_PERIODIC_X || d->bc == SL_BC_PERIODIC_Y)))
        return SL_E_INVALID;
    if (d->form != SL_FORM_ADVECTIVE && d->form != SL_FORM_CONSERVATIVE) return SL_E_INVALID;
    if (d->precision != SL_PREC_FP64 &&
        !((d->precision == SL_PREC_FP32_REFINED || d->precision == SL_PREC_BF16_REFINED) && d->dim == 2 &&
          n <= kMax2DFull))
        return SL_E_INVALID;
    if (!(d->x1 > d->x0) || (d->dim == 2 && !(d->y1 > d->y0))) return SL_E_INVALID;
    if (!std::isfinite(d->x0) || !std::isfinite(d->x1)) return SL_E_INVALID;

    sl_mesh* m = new (std::nothrow) sl_mesh();
    if (!m) return SL_E_NOMEM;
    m->bump = tl_bump;
    m->dim = d->dim; m->kx = d->kx; m->ky = d->ky; m->n = n;
    m->nd = d->dim == 1 ? n : n * n;
    m->K = d->kx * d->ky;
    m->family = d->nodes; m->bc = d->bc; m->form = d->form; m->precision = d->precision;
    m->x0 = d->x0; m->x1 = d->x1; m->y0 = d->y0; m->y1 = d->y1;
    m->dx = (d->x1 - d->x0) / d->kx;
    m->dy = d->dim == 2 ? (d->y1 - d->y0) / d->ky : 1.0;
    const size_t nf = (size_t)m->K * m->nd;
    if (!all_finite(d->u0, nf)) { delete m; return SL_E_NONFINITE; }
    if (!build_tables(m->family, n, &m->T)) { delete m; return SL_E_INVALID; }
    m->off = tab_offsets(m->dim, n);

    if (d->stream) { m->stream = (hipStream_t)d->stream; m->own_stream = false; }
    else {
        if (hipStreamCreateWithFlags(&m->stream, hipStreamNonBlocking) != hipSuccess) { delete m; return SL_E_DEVICE; }
        m->own_stream = true;
    }
    const BufSizes z = buffer_sizes(m->dim, m->kx, m->ky, n);
    m->nblocks = z.nblocks;
    m->nslice = 1;
    bool ok = dalloc(m, &m->phi, z.nf) && dalloc(m, &m->phi2, z.nf) && dalloc(m, &m->phihat, z.nf) &&
              dalloc(m, &m->rec, z.nrec) && dalloc(m, &m->aN, z.nf * m->dim) && dalloc(m, &m->aM, z.ncoef) &&
              dalloc(m, &m->divN, z.nf) && dalloc(m, &m->divM, z.nf) && dalloc(m, &m->vface, z.nvf) &&
              dalloc(m, &m->tab, z.ntab) && dalloc(m, &m->stat_part, z.nstat) && dalloc(m, &m->flag_part, z.nflag) &&
              dalloc(m, &m->vdeg_d, 1);
    if (!ok) { release(m); delete m; return SL_E_NOMEM; }

    std::vector<double> tab(m->off.total, 0.0);
    for (int j = 0; j < n; ++j) {
        tab[m->off.xi + j] = m->T.xi[j];
        tab[m->off.w + j] = m->T.w[j];
        tab[m->off.l0 + j] = m->T.l0[j];
        tab[m->off.l1 + j] = m->T.l1[j];
        for (int k = 0; k < n; ++k) {
            tab[m->off.tinv + j * n + k] = m->T.Tinv[j * n + k];
            tab[m->off.dmat + j * n + k] = m->T.D[j * n + k];
        }
    }
    if (m->dim == 2) {
        for (int j = 0; j < n; ++j) tab[m->off.lam + j] = m->T.lam[j];
        if (!build_boundary_tables(m->T, &tab[m->off.cbp], &tab[m->off.softs], &tab[m->off.zmh],
                                   &tab[m->off.zms])) {
            release(m);
            delete m;
            return SL_E_INVALID;
        }
    }
    hipError_t e1 = hipMemcpyAsync(m->tab, tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice, m->stream);
    hipError_t e2 = hipMemcpyAsync(m->phi, d->u0, nf * sizeof(double), hipMemcpyHostToDevice, m->stream);
    hipError_t e3 = hipMemsetAsync(m->stat_part, 0, (size_t)m->nblocks * kStatSlots * sizeof(double), m->stream);
    hipError_t e4 = hipMemsetAsync(m->flag_part, 0, (size_t)2 * m->nblocks * sizeof(int32_t), m->stream);
    hipError_t e5 = hipStreamSynchronize(m->stream);
    if (e1 || e2 || e3 || e4 || e5) { release(m); delete m; return SL_E_DEVICE; }
    *out = m;
    return SL_OK;
}

sl_status sl_destroy_mesh(sl_mesh* m)
{
    const ApiHold hold;
    if (!m) return SL_E_INVALID;
    (void)hipStreamSynchronize(m->stream);
    release(m);
    delete m;
    return SL_OK;
}

sl_status sl_mesh_bytes(const sl_mesh_desc* d, int32_t ghost_rows, size_t* bytes)
{
    if (!d || !bytes || (d->dim != 1 && d->dim != 2) || d->kx < 1 || d->ky < 1 || ghost_rows < 0) return SL_E_INVALID;
    if (d->orders) {
        MixedPlan P;
        if (!mixed_plan(d, &P)) return SL_E_INVALID;
        *bytes = mixed_bytes(d, P);
        return SL_OK;
    }
    const int n = d->order + 1;
    if (d->order < 1 || n > (d->dim == 1 ? kMax1D : kMax2D) || (d->dim == 1 && d->ky != 1)) return SL_E_INVALID;
    if ((int64_t)d->kx * d->ky > (1 << 26)) return SL_E_INVALID;
    const BufSizes z = buffer_sizes(d->dim, d->kx, d->ky, n);
    const size_t ng = d->dim == 1 ? 2 : (size_t)2 * n * (d->kx + d->ky);
    const size_t dbl = 3 * z.nf + z.nrec + z.nf * d->dim + z.ncoef + 2 * z.nf + z.nvf + z.ntab + z.nstat +
                       (d->bc != SL_BC_PERIODIC ? ng * ghost_rows : 0);
    *bytes = dbl * sizeof(double) + (z.nflag + 1) * sizeof(int32_t);
    return SL_OK;
}

sl_status sl_set_velocity(sl_mesh* m, const double* a, const double* div_a)
{
    const ApiHold hold;
    if (!m || !a) return SL_E_INVALID;
    if (m->mixed) return set_velocity_mixed(m, a, div_a);
    const size_t nf = (size_t)m->K * m->nd;
    if (!all_finite(a, nf * m->dim)) return SL_E_NONFINITE;
    if (div_a && !all_finite(div_a, nf)) return SL_E_NONFINITE;
    double am[2] = {0.0, 0.0};
    for (int c = 0; c < m->dim; ++c)
        for (size_t i = 0; i < nf; ++i) am[c] = std::max(am[c], std::fabs(a[c * nf + i]));
    if (hipMemcpyAsync(m->aN, a, nf * m->dim * sizeof(double), hipMemcpyHostToDevice, m->stream)) return SL_E_DEVICE;
    if (div_a && hipMemcpyAsync(m->divN, div_a, nf * sizeof(double), hipMemcpyHostToDevice, m->stream))
        return SL_E_DEVICE;
    if (hipMemsetAsync(m->vdeg_d, 0, sizeof(int32_t), m->stream)) return SL_E_DEVICE;
    const int cons = m->form == SL_FORM_CONSERVATIVE;
    int rc = m->dim == 1
                 ? launch_prep1d(m->n, m->K, m->bc == SL_BC_PERIODIC, div_a != nullptr, m->aN, m->aM, m->divN,
                                 m->divM, m->aM + (size_t)m->K * m->n, m->aM + (size_t)m->K * (m->n + 4), m->vface,
                                 m->tab, m->dx, cons, std::max(am[0], am[1]), m->vdeg_d, m->stream)
                 : launch_prep2d(m->n, m->K, div_a != nullptr, cons, m->aN, m->aM, m->divN, m->divM, m->tab, m->dx,
                                 m->dy, std::max(am[0], am[1]), m->vdeg_d, m->stream);
    if (!rc && m->dim == 2)
        rc = launch_facevel2d(m->n, m->kx, m->ky, periodic_mask(m->bc), m->aN, m->tab,
                              1e-12 * std::max(am[0], am[1]), m->vface, m->stream);
    int32_t vdeg = m->n - 1;
    if (rc || hipMemcpyAsync(&vdeg, m->vdeg_d, sizeof(int32_t), hipMemcpyDeviceToHost, m->stream) ||
        hipStreamSynchronize(m->stream))
        return SL_E_DEVICE;
    m->vdeg = vdeg;
    m->amax[0] = am[0];
    m->amax[1] = am[1];
    m->has_velocity = true;
    return SL_OK;
}

int32_t sl_ghost_count(const sl_mesh* m)
{
    if (!m) return 0;
    return m->dim == 1 ? 2 : 2 * m->ky * m->n + 2 * m->kx * m->n;
}

sl_status sl_set_ghost(sl_mesh* m, const double* g, int32_t nrows)
{
    const ApiHold hold;
    if (!m) return SL_E_INVALID;
    if (m->bc == SL_BC_PERIODIC) return SL_E_STATE;
    if (!g || nrows < 1) return SL_E_INVALID;
    const size_t per = (size_t)sl_ghost_count(m), cnt = per * nrows;
    // the values that are read must be finite: every side of a GHOST mesh,
    // the bottom and top sides of SL_BC_PERIODIC_X, the left and right
    // sides of SL_BC_PERIODIC_Y (row layout: left, right, bottom, top)
    const size_t lr = m->dim == 2 ? (size_t)2 * m->ky * m->n : per;
    const size_t lo = m->bc == SL_BC_PERIODIC_X ? lr : 0, hi = m->bc == SL_BC_PERIODIC_Y ? lr : per;
    for (int32_t r = 0; r < nrows; ++r)
        if (!all_finite(g + r * per + lo, hi - lo)) return SL_E_NONFINITE;
    if (hipStreamSynchronize(m->stream)) return SL_E_DEVICE;
    dfree(m, m->ghost);
    if (!dalloc(m, &m->ghost, cnt)) { m->ghost_rows = 0; return SL_E_NOMEM; }
    if (hipMemcpyAsync(m->ghost, g, cnt * sizeof(double), hipMemcpyHostToDevice, m->stream)) return SL_E_DEVICE;
    m->ghost_rows = nrows;
    m->ghost_step = 0;
    return SL_OK;
}

double sl_max_dt(const sl_mesh* m, double cfl)
{
    if (!m || !m->has_velocity || !(cfl > 0)) return 0.0;
    const double gap = m->T.xi[0];
    double dt = INFINITY;
    if (m->amax[0] > 0) dt = std::min(dt, gap * m->dx / m->amax[0]);
    if (m->dim == 2 && m->amax[1] > 0) dt = std::min(dt, gap * m->dy / m->amax[1]);
    if (!std::isfinite(dt)) dt = 0.0;
    return dt * cfl;
}


}  // extern "C"

namespace {

// validation of a step (before any launch; the mesh is unchanged on error)
sl_status step_check(const sl_mesh* m, double dt, int32_t nsteps, const sl_step_opts& opt)
{
    if (!(dt > 0) || !std::isfinite(dt) || nsteps < 0) return SL_E_INVALID;
    if (!step_opts_valid(opt)) return SL_E_INVALID;
    if (m->mixed && opt.iface != SL_IFACE_INTERP) return SL_E_INVALID;
    if (!m->has_velocity) return SL_E_STATE;
    if (m->bc != SL_BC_PERIODIC && m->ghost_rows < 1) return SL_E_STATE;
    // time-step restriction: particles may not cross the element-edge gap
    // dt <= gap dx / max|a| (the paper's condition admits equality; a relative
    // 1e-12 slack absorbs the rounding of dt computed at the limit)
    const double gap = m->T.xi[0];
    if (m->amax[0] * dt > gap * m->dx * (1.0 + 1e-12)) return SL_E_CFL;
    if (m->dim == 2 && m->amax[1] * dt > gap * m->dy * (1.0 + 1e-12)) return SL_E_CFL;
    // the rows of the 1D KKT system must be independent: n >= number of rows
    const int rows = ((opt.constraints & SL_C_BOUNDARY) ? 2 : 0) + ((opt.constraints & SL_C_MASS) ? 1 : 0) +
                     ((opt.constraints & SL_C_ENERGY) ? 1 : 0);
    if (rows > m->nd) return SL_E_INVALID;
    // 2D HARD: the mass and energy rows are imposed inside null(C_B), of
    // dimension n^2 - (4n - 4) = (n - 2)^2; more rows than that have no
    // exact solution (SOFT, the stacked least squares, always has one)
    if (m->dim == 2 && opt.mode == SL_MODE_HARD && (opt.constraints & SL_C_BOUNDARY) &&
        rows - 2 > (m->n - 2) * (m->n - 2))
        return SL_E_INVALID;
    // above 16 nodes per direction a 2D step takes boundary rows only (the
    // mass and energy rows run one lane per node)
    if (m->dim == 2 && !m->mixed && m->n > kMax2DFull && (opt.constraints & (SL_C_MASS | SL_C_ENERGY)))
        return SL_E_INVALID;
    return SL_OK;
}

// launch arguments of a uniform 2D mesh's steps, but the per-step fields
void args2d(const sl_mesh* m, double dt, const sl_step_opts& opt, Step2DArgs* Bp)
{
    Step2DArgs& B = *Bp;
    std::memset(&B, 0, sizeof(B));
    rk_tableau(opt.rk, &B.rk);
    B.aN = m->aN; B.aM = m->aM; B.divN = m->divN; B.divM = m->divM; B.vface = m->vface; B.tab = m->tab;
    B.rec = m->rec; B.phihat = m->phihat;
    B.flag_part = m->flag_part; B.stat_part = m->stat_part; B.nblk = m->nblocks; B.vdeg = m->vdeg;
    B.kx = m->kx; B.ky = m->ky; B.K = m->K; B.periodic = periodic_mask(m->bc);
    B.cons = m->form == SL_FORM_CONSERVATIVE; B.cmask = opt.constraints; B.mode = opt.mode;
    B.refine = 60;  // cap on defect-correction sweeps of the remap solve
    B.precision = m->precision;
    B.targets = (opt.constraints & (SL_C_MASS | SL_C_ENERGY)) != 0;
    // volume terms of the balance laws: advective form for mass and
    // energy, conservative form for energy only
    B.vol = B.targets && (B.cons ? (opt.constraints & SL_C_ENERGY) != 0 : 1);
    B.rstride = (B.targets ? 12 * m->n + 3 : 4 * m->n) + (opt.iface == SL_IFACE_BACKTRACK ? 4 * m->n : 0);
    // from n = 12 on one element fills a 256-lane block only to 66% or
    // less: the advect (FP64) takes the block of the fewest whole waves
    // that hold one element instead (192 lanes at n = 13; measured 13%
    // faster).  A block then still holds one element, so the per-block
    // partials stay sized as they are.
    B.bs = (m->n >= 12 && m->precision == SL_PREC_FP64) ? 1 : 0;
    B.sumW = 0.0;
    for (int j = 0; j < m->n; ++j)
        for (int i = 0; i < m->n; ++i) B.sumW += m->dx * m->dy * m->T.w[i] * m->T.w[j];
    B.emaxit = opt.energy_maxit; B.etol = opt.energy_tol;
    B.iface = opt.iface;
    B.dx = m->dx; B.dy = m->dy;
    B.invdx = 1.0 / m->dx; B.invdy = 1.0 / m->dy; B.dt = dt;
    B.vzero = 1e-12 * std::max(m->amax[0], m->amax[1]);
}

// launch arguments of a 1D mesh's steps, but the per-step fields; false if
// the constant block of the KKT system is singular
bool args1d(const sl_mesh* m, double dt, const sl_step_opts& opt, Step1DArgs* Ap)
{
    Step1DArgs& A = *Ap;
    std::memset(&A, 0, sizeof(A));
    if (!step1d_setup(m->T, m->n, m->dx, m->bc == SL_BC_PERIODIC, m->form == SL_FORM_CONSERVATIVE, opt,
                      m->amax[0], &A))
        return false;
    A.aN = m->aN; A.aM = m->aM; A.divN = m->divN; A.divM = m->divM; A.vface = m->vface; A.tab = m->tab;
    A.aM4 = m->aM + (size_t)m->K * m->n;
    A.divM4 = m->aM + (size_t)m->K * (m->n + 4);
    A.rec = m->rec; A.phihat = m->phihat;
    A.flag_part = m->flag_part; A.stat_part = m->stat_part; A.nblk = m->nblocks; A.vdeg = m->vdeg;
    A.K = m->K;
    A.dt = dt;
    return true;
}

// the per-step fields of the next step: phi^n, phi^{n+1} and the ghost rows
// at t^n and t^{n+1}
template <typename Args>
void step_fields(const sl_mesh* m, Args* A)
{
    if (m->bc != SL_BC_PERIODIC) {
        const long r0 = std::min<long>(m->ghost_step, m->ghost_rows - 1);
        const long r1 = std::min<long>(m->ghost_step + 1, m->ghost_rows - 1);
        A->gnow = m->ghost + r0 * sl_ghost_count(m);
        A->gnext = m->ghost + r1 * sl_ghost_count(m);
    } else {
        A->gnow = A->gnext = m->vface;  // unused for periodic meshes (valid address)
    }
    A->phi = m->phi;
    A->phi_out = m->phi2;
}

// a step launched: the new field becomes phi^n
void commit(sl_mesh* m, double dt)
{
    std::swap(m->phi, m->phi2);
    m->t += dt;
    m->steps += 1;
    m->ghost_step += 1;
}

}  // namespace

sl_status sl::step_prepare(sl_mesh* m, double dt, const sl_step_opts& opt, StepLaunch* L)
{
    const sl_status rc = step_check(m, dt, 1, opt);
    if (rc != SL_OK) return rc;
    L->dim = m->dim;
    L->n = m->n;
    L->variant = -1;
    if (m->mixed || m->profiling) return SL_OK;
    if (m->dim == 1) {
        if (!args1d(m, dt, opt, &L->a1)) return SL_E_INVALID;
        step_fields(m, &L->a1);
        L->variant = advect1d_variant(m->n, L->a1);
        L->adv_blocks = advect1d_blocks(m->n, m->K);
        L->con_blocks = constrain1d_blocks(m->K);
        return SL_OK;
    }
    args2d(m, dt, opt, &L->a2);
    step_fields(m, &L->a2);
    // batched: boundary rows, interpolated face values, and a constrain with
    // no more chunks than the per-block partials hold (from n = 4 on)
    if (L->a2.targets || opt.iface != SL_IFACE_INTERP || m->n < 4) return SL_OK;
    L->variant = L->a2.precision * 4 + L->a2.bs;
    L->adv_blocks = advect2d_blocks(m->n, L->a2.bs, m->K);
    L->con_blocks = constrain2d_chunks(m->n, m->K);
    if (L->adv_blocks > m->nblocks || L->con_blocks > m->nblocks) L->variant = -1;
    return SL_OK;
}

void sl::step_commit(sl_mesh* m, double dt) { commit(m, dt); }

extern "C" {

sl_status sl_step(sl_mesh* m, double dt, int32_t nsteps, const sl_step_opts* o)
{
    const ApiHold hold;
    if (!m) return SL_E_INVALID;
    sl_step_opts opt = {4, SL_C_BOUNDARY, SL_MODE_HARD, 50, 3, SL_IFACE_INTERP, 1e-8};
    if (o) opt = *o;
    const sl_status rc = step_check(m, dt, nsteps, opt);
    if (rc != SL_OK) return rc;

    if (m->mixed) return step_mixed(m, dt, nsteps, opt);
    if (m->dim == 2) {
        Step2DArgs B;
        args2d(m, dt, opt, &B);
        for (int s = 0; s < nsteps; ++s) {
            step_fields(m, &B);
            if (opt.iface == SL_IFACE_BACKTRACK) {
                ev_begin(m, KER_BT2D, true);
                if (launch_backtrace2d(m->n, B, m->stream)) return SL_E_DEVICE;
                ev_end(m, KER_BT2D, true);
            }
            if (B.targets) {
                ev_begin(m, KER_TGT2D, true);
                if (launch_targets2d(m->n, B, m->stream)) return SL_E_DEVICE;
                ev_end(m, KER_TGT2D, true);
            }
            ev_begin(m, KER_ADV2D, true);
            if (launch_advect2d(m->n, B, m->stream)) return SL_E_DEVICE;
            ev_end(m, KER_ADV2D, true);
            ev_begin(m, KER_CON2D, true);
            if (launch_constrain2d(m->n, B, m->stream)) return SL_E_DEVICE;
            ev_end(m, KER_CON2D, true);
            commit(m, dt);
        }
        return SL_OK;
    }

    Step1DArgs A;
    if (!args1d(m, dt, opt, &A)) return SL_E_INVALID;
    for (int s = 0; s < nsteps; ++s) {
        step_fields(m, &A);
        ev_begin(m, KER_ADV1D, true);
        if (launch_advect1d(m->n, A, m->stream)) return SL_E_DEVICE;
        ev_end(m, KER_ADV1D, true);
        ev_begin(m, KER_CON1D, true);
        if (launch_constrain1d(m->n, A, m->stream)) return SL_E_DEVICE;
        ev_end(m, KER_CON1D, true);
        commit(m, dt);
    }
    return SL_OK;
}

}  // extern "C"

namespace {

// sl_read; sync = false when the caller knows the mesh's work is done
// (its stream may hold later work of other meshes)
sl_status read_impl(sl_mesh* m, double* u_out, sl_stats* st, bool sync)
{
    if (sync && hipStreamSynchronize(m->stream)) return SL_E_DEVICE;
    const size_t nf = m->mixed ? m->dofs : (size_t)m->K * m->nd;
    std::vector<double> host;
    double* dst = u_out;
    if (!dst && st) { host.resize(nf); dst = host.data(); }
    if (dst && m->mixed) {
        std::vector<double> dev(nf);
        if (hipMemcpy(dev.data(), m->phi, nf * sizeof(double), hipMemcpyDeviceToHost)) return SL_E_DEVICE;
        for (int e = 0; e < m->K; ++e)
            std::memcpy(dst + m->uoff[e], &dev[m->doff[e]], sizeof(double) * m->orders[e] * m->orders[e]);
    } else if (dst && hipMemcpy(dst, m->phi, nf * sizeof(double), hipMemcpyDeviceToHost)) {
        return SL_E_DEVICE;
    }
    const int nb = m->nslice * m->nblocks;
    std::vector<double> sp((size_t)nb * kStatSlots);
    std::vector<int32_t> fp((size_t)2 * nb);
    if (hipMemcpy(sp.data(), m->stat_part, sp.size() * sizeof(double), hipMemcpyDeviceToHost)) return SL_E_DEVICE;
    if (hipMemcpy(fp.data(), m->flag_part, fp.size() * sizeof(int32_t), hipMemcpyDeviceToHost)) return SL_E_DEVICE;
    int flags = 0;
    for (int32_t f : fp) flags |= f;
    double rb = 0, rm = 0, re = 0, pic = 0, swsum = 0, swmax = 0, rres = 0;
    for (int b = 0; b < nb; ++b) {
        rb = std::max(rb, sp[b * kStatSlots + 0]);
        rm = std::max(rm, sp[b * kStatSlots + 1]);
        re = std::max(re, sp[b * kStatSlots + 2]);
        pic = std::max(pic, sp[b * kStatSlots + 3]);
        swsum += sp[b * kStatSlots + 4];
        swmax = std::max(swmax, sp[b * kStatSlots + 5]);
        rres = std::max(rres, sp[b * kStatSlots + 6]);
    }
    const int64_t dsteps = m->steps - m->steps_read;
    if (st) {
        std::memset(st, 0, sizeof(*st));
        st->t = m->t;
        st->steps = m->steps;
        // mass and energy on the device, the block sums into phihat (free
        // between steps), summed here in a fixed order
        struct Seg {
            const double* phi;
            size_t nf;
            int n;
            const double* w;
        };
        std::vector<Seg> seg;
        if (m->mixed)
            for (int b = 0; b < m->nbk; ++b)
                seg.push_back({m->phi + m->bOff[b], (size_t)m->bK[b] * m->bn[b] * m->bn[b], m->bn[b],
                               m->tab + m->tabOff[b] + tab_offsets(2, m->bn[b]).w});
        else
            seg.push_back({m->phi, nf, m->n, m->tab + m->off.w});
        size_t np = 0;
        for (const Seg& g : seg) {
            if (g.nf && launch_moments(g.phi, g.nf, g.n, m->dim, g.w, m->phihat + 2 * np, m->stream)) return SL_E_DEVICE;
            np += g.nf ? (size_t)moments_blocks(g.nf) : 0;
        }
        std::vector<double> part(2 * np);
        if (np && (hipMemcpyAsync(part.data(), m->phihat, part.size() * sizeof(double), hipMemcpyDeviceToHost,
                                  m->stream) != hipSuccess ||
                   hipStreamSynchronize(m->stream) != hipSuccess))
            return SL_E_DEVICE;
        double M = 0, E = 0;
        for (size_t k = 0; k < np; ++k) {
            M += part[2 * k];
            E += part[2 * k + 1];
        }
        const double h = m->dim == 2 ? m->dx * m->dy : m->dx;
        M *= h;
        E *= h;
        st->mass = M;
        st->energy = E;
        st->resid_boundary = rb;
        st->resid_mass = rm;
        st->resid_energy = re;
        st->max_picard = (int32_t)pic;
        st->flags = flags;
        st->vel_terms = vel_terms_used(m);
        st->refine_resid = rres;
        st->remap_sweeps_max = (int32_t)swmax;
        st->remap_sweeps_mean = dsteps > 0 ? swsum / ((double)dsteps * m->K) : 0.0;
    }
    m->steps_read = m->steps;
    (void)hipMemsetAsync(m->stat_part, 0, sp.size() * sizeof(double), m->stream);
    (void)hipMemsetAsync(m->flag_part, 0, fp.size() * sizeof(int32_t), m->stream);
    if (hipStreamSynchronize(m->stream)) return SL_E_DEVICE;
    if (flags & FLAG_NONFINITE) return SL_E_NONFINITE;
    if (flags & FLAG_SINGULAR) return SL_E_SINGULAR;
    if (flags & FLAG_NOCONV) return SL_E_NOCONV;
    return SL_OK;
}

}  // namespace

sl_status sl::read_settled(sl_mesh* m, double* u_out, sl_stats* st)
{
    return m ? read_impl(m, u_out, st, false) : SL_E_INVALID;
}

extern "C" {

sl_status sl_read(sl_mesh* m, double* u_out, sl_stats* st)
{
    const ApiHold hold;
    if (!m) return SL_E_INVALID;
    return read_impl(m, u_out, st, true);
}

sl_status sl_device_field(sl_mesh* m, double** d_phi, void** stream)
{
    if (!m) return SL_E_INVALID;
    if (d_phi) *d_phi = m->phi;
    if (stream) *stream = (void*)m->stream;
    return SL_OK;
}

sl_status sl_set_profiling(sl_mesh* m, int32_t enable)
{
    const ApiHold hold;
    if (!m) return SL_E_INVALID;
    (void)hipStreamSynchronize(m->stream);
    for (int k = 0; k < KER_COUNT; ++k) {
        for (hipEvent_t e : m->pending[k]) (void)hipEventDestroy(e);
        m->pending[k].clear();
        m->ktime[k] = 0.0;
        m->kcount[k] = 0;
    }
    m->profiling = enable != 0;
    return SL_OK;
}

sl_status sl_kernel_time(sl_mesh* m, int32_t which, double* total_ms, int64_t* launches)
{
    const ApiHold hold;
    if (!m || which < 0 || which >= KER_COUNT) return SL_E_INVALID;
    if (hipStreamSynchronize(m->stream)) return SL_E_DEVICE;
    auto& v = m->pending[which];
    for (size_t i = 0; i + 1 < v.size(); i += 2) {
        float ms = 0.f;
        if (hipEventElapsedTime(&ms, v[i], v[i + 1]) == hipSuccess) m->ktime[which] += ms;
        m->kcount[which] += 1;
        (void)hipEventDestroy(v[i]);
        (void)hipEventDestroy(v[i + 1]);
    }
    v.clear();
    if (total_ms) *total_ms = m->ktime[which];
    if (launches) *launches = m->kcount[which];
    return SL_OK;
}

sl_status sl_bucket_stats(sl_mesh* m, int32_t bucket, int32_t* n, int32_t* count, int32_t* vel_terms,
                          double* sweeps_mean)
{
    const ApiHold hold;
    if (!m || bucket < 0 || bucket >= (m->mixed ? m->nbk : 1)) return SL_E_INVALID;
    if (hipStreamSynchronize(m->stream)) return SL_E_DEVICE;
    const int b = m->mixed ? bucket : 0;
    const int K = m->mixed ? m->bK[b] : m->K;
    std::vector<double> sp((size_t)m->nblocks * kStatSlots);
    if (hipMemcpy(sp.data(), m->stat_part + (size_t)b * m->nblocks * kStatSlots, sp.size() * sizeof(double),
                  hipMemcpyDeviceToHost))
        return SL_E_DEVICE;
    double sw = 0.0;
    for (int k = 0; k < m->nblocks; ++k) sw += sp[(size_t)k * kStatSlots + 4];
    const int64_t dsteps = m->steps - m->steps_read;
    if (n) *n = m->mixed ? m->bn[b] : m->n;
    if (count) *count = K;
    if (vel_terms) *vel_terms = m->mixed ? m->bdeg[b] + 1 : vel_terms_used(m);
    if (sweeps_mean) *sweeps_mean = dsteps > 0 ? sw / ((double)dsteps * K) : 0.0;
    return SL_OK;
}

}  // extern "C"
