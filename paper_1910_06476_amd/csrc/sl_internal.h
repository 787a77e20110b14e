// Internal declarations shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/sl.h"

namespace sl {

constexpr int kMaxTableN = 32;
constexpr int kMax1D = 17;  // nodes per element in 1D (order 16)
constexpr int kMax2D = 17;  // nodes per direction in 2D (order 16)
// Above 16 nodes per direction (n^2 > 256 particles) a 2D element takes a
// block of its own in the advect, in FP64 with boundary rows only
constexpr int kMax2DFull = 16;
constexpr int kMaxBuckets = 16;  // distinct orders of a mixed-order mesh

struct Tables {
    int n;
    double xi[kMaxTableN], w[kMaxTableN], lam[kMaxTableN];
    double l0[kMaxTableN], l1[kMaxTableN];
    double D[kMaxTableN * kMaxTableN];
    double Tinv[kMaxTableN * kMaxTableN];
};

// Periodicity of a boundary condition as a mask for the kernels: bit 0 the
// left and right sides wrap, bit 1 the bottom and top sides (1D meshes use
// bit 0 only).
inline int periodic_mask(int bc)
{
    return bc == SL_BC_PERIODIC ? 3 : bc == SL_BC_PERIODIC_X ? 1 : bc == SL_BC_PERIODIC_Y ? 2 : 0;
}

bool node_rule(int family, int n, double* xi, double* w);
bool invert(int n, const double* A, double* Ainv);
bool build_tables(int family, int n, Tables* T);

// Device table layout (doubles), per mesh.  1D and 2D share the head.
struct TabOff {
    int xi, w, l0, l1, tinv, dmat;   // n, n, n, n, n*n, n*n
    int lam, cbp, softs;              // 2D: lambda (n), Qhard (4n x 4n), Qsoft (4n x 4n)
    int zmh, zms;                     // 2D: projected mass rows (n^2 each)
    int total;
};
TabOff tab_offsets(int dim, int n);

// Explicit Runge-Kutta tableau, with the distinct abscissae and their
// summed weights (the quadrature the tableau induces on a time integral).
struct RKTab {
    int s, nq;
    double a[4][4], b[4], c[4];
    double cu[4], bu[4];
};
bool rk_tableau(int order, RKTab* T);

// timed kernels (sl_kernel_time): the uniform-mesh kernels, the whole step of
// a mixed-order mesh (KER_ADV2D), per bucket b its advect (KER_MIX_ADV + b)
// and constrain (KER_MIX_CON + b) launches, and the uniform 2D mesh's
// targets (KER_TGT2D) and face backtrace (KER_BT2D) launches
enum {
    KER_ADV1D = 0, KER_CON1D = 1, KER_ADV2D = 2, KER_CON2D = 3,
    KER_MIX_ADV = 4, KER_MIX_CON = 4 + kMaxBuckets, KER_TGT2D = 4 + 2 * kMaxBuckets, KER_BT2D = KER_TGT2D + 1,
    KER_COUNT = KER_BT2D + 1
};
enum { FLAG_NONFINITE = 1, FLAG_CONTAIN = 2, FLAG_SINGULAR = 4, FLAG_NOCONV = 8 };

// Per-block statistics slots: [resid_boundary, resid_mass, resid_energy,
// max_picard] from the constraint kernels, [remap sweeps summed over
// elements, max sweeps, max final relative correction] from the 2D advect
constexpr int kStatSlots = 7;

// 1D per-element record (doubles), written by the advect kernel and read by
// the constrain kernel of the element and of its two neighbours:
//   [0] T0, [1] T1          edge values at t^{n+1} (traces of phihat, or
//                           backtraced values at upwind edges)
//   [2] S1_L, [3] S1_R      sum_q b_q (v_q - c) over the RK abscissae of the
//                           values v_q at the left / right edge (upwind
//                           edges only, else zero)
//   [4] S2_L, [5] S2_R      sum_q b_q (v_q - c)^2
//   [6] M                   M^n + dt * volume term of the mass balance
//   [7] Ed                  sum W (phi^n - c)^2 + dt * volume term of the
//                           deviation energy balance
//   [8] c                   the element's mean at t^n, M^n / sum W
constexpr int kRec1 = 9;

struct Step1DArgs {
    // fields
    const double* phi;     // [K][n] phi^n
    double* phihat;        // [K][n] remapped
    double* rec;           // [K][kRec1] per-element record
    double* phi_out;       // [K][n] phi^{n+1}
    // velocity
    const double* aN;      // nodal velocity
    const double* aM;      // Chebyshev coefficients of the velocity
    const double* divN;    // nodal divergence
    const double* divM;    // Chebyshev coefficients of the divergence
    const double* aM4;     // [K][4] the first four of aM, contiguous (a short series reads only these)
    const double* divM4;   // [K][4] the first four of divM
    const double* vface;   // [K+1] face velocity
    const double* tab;
    const double* gnow;    // ghost row at t^n (2 values) or null
    const double* gnext;   // ghost row at t^{n+1}
    int32_t* flag_part;    // [2][nblk]
    double* stat_part;     // [nblk][kStatSlots]
    int nblk;
    int vdeg;              // mesh-wide effective degree of the velocity series
    int K, periodic, cons, cmask, mode, emaxit, vol, targets;
    int iface;             // SL_IFACE_*: edge values by interpolation or backtracking
    double dx, invdx, dt, etol, vzero;
    double sumW;  // sum of the element's quadrature weights W = dx w
    double g00, g01, g11, g02, g12, g22;  // constant Gram entries of rows l(0), l(1), W
    double g3i[9];  // inverse of the constant 3x3 block of the launch's system (rows l(0), l(1), W;
                    // inactive rows as identity; + I in SOFT), row-major
    RKTab rk;
};

// Ordering of the library's graph captures against its own calls that may
// allocate, free or synchronise device memory from other host threads: a
// capture that such a call disturbs fails (the stream's capture is
// invalidated, or the call is refused while a capture is active), so
// distinct meshes used from several threads could see spurious device
// errors.  ApiHold is taken (shared, nestable within a thread) by the public
// calls that make such calls; CaptureHold (exclusive) by a capture, which
// only enqueues launches; it gives up the thread's own shared hold meanwhile.
struct ApiHold {
    ApiHold();
    ~ApiHold();
};
struct CaptureHold {
    CaptureHold();
    ~CaptureHold();
    int saved;
};

// Per-kernel timing: the pair of events that the next timed launch made on
// this thread records itself, with the dispatch's own start and end
// timestamps (the interval a kernel trace reports, free of the packets and
// fences that events recorded on the stream around it add), or none.  Set
// just before one launch and taken by it.
struct LaunchEvents {
    hipEvent_t start = nullptr, stop = nullptr;
};
extern thread_local LaunchEvents tl_timed_launch;

// A block of device memory that meshes created on this thread carve their
// buffers from (256-byte aligned, in order) instead of allocating them; the
// block's owner frees it after the meshes are destroyed.  Set around a
// mesh's creation and set-up by the request loop; null elsewhere.
struct BumpBlock {
    char* base = nullptr;
    size_t size = 0, used = 0;
};
extern thread_local BumpBlock* tl_bump;

// Mass and energy partial sums of nf nodes of order n (sl_moments.hip):
// moments_blocks(nf) blocks each write (sum w phi, sum w phi^2) to
// part[2b], part[2b + 1]; w is the device copy of the node weights.
int moments_blocks(size_t nf);
int launch_moments(const double* phi, size_t nf, int n, int dim, const double* w, double* part, hipStream_t s);

template <typename F, typename... Args>
inline void launch_timed(F kernel, dim3 grid, dim3 block, uint32_t shm, hipStream_t s, Args... args)
{
    const LaunchEvents ev = tl_timed_launch;
    if (ev.start) {
        tl_timed_launch = LaunchEvents{};
        hipExtLaunchKernelGGL(kernel, grid, block, shm, s, ev.start, ev.stop, 0u, args...);
    } else {
        hipLaunchKernelGGL(kernel, grid, block, shm, s, args...);
    }
}

// Step options within their documented ranges.
bool step_opts_valid(const sl_step_opts& opt);
// Launch constants of a 1D step that do not depend on the buffers: tableau,
// options, the Gram entries of the rows l(0), l(1), W and the inverse of
// their constant 3x3 block, sum W, and the stagnation threshold 1e-12 amax
// (amax = max |a| over the nodes).  False if that block is singular.
bool step1d_setup(const Tables& T, int n, double dx, int periodic, int cons, const sl_step_opts& opt, double amax,
                  Step1DArgs* A);

// Batched 1D steps: one launch of each kernel steps several meshes, block
// offsets start[0..nreq] (start[0] = 0, start[nreq] = nblocks) and the
// members' arguments As in device memory; A0 a host copy of one member's.
// The members share n and advect1d_variant; n >= 2.
int advect1d_variant(int n, const Step1DArgs& A);
int advect1d_blocks(int n, int K);
int constrain1d_blocks(int K);
int launch_advect1d_batch(int n, const Step1DArgs& A0, const Step1DArgs* As, const int* start, int nreq,
                          int nblocks, hipStream_t s);
int launch_constrain1d_batch(int n, const Step1DArgs* As, const int* start, int nreq, int nblocks, hipStream_t s);

// vscale: mesh-wide max |a|, the floor of the noise threshold of the
// velocity series' effective degree
int launch_prep1d(int n, int K, int periodic, int has_div, const double* aN, double* aM, double* divN,
                  double* divM, double* aM4, double* divM4, double* vface, const double* tab, double dx, int cons,
                  double vscale, int* vdeg, hipStream_t s);
int launch_advect1d(int n, const Step1DArgs& A, hipStream_t s);
int launch_constrain1d(int n, const Step1DArgs& A, hipStream_t s);
int blocks1d(int n, int K);

struct Step2DArgs {
    const double* phi;     // [K][n^2] phi^n
    double* phihat;        // [K][n^2] remapped
    double* rec;           // [K][rstride] edge traces of phihat (4n); with targets also the
                           // upwind stage sums about the element's mean c (2 x 4n), the local
                           // mass and deviation energy parts (2) and c; with backtracking,
                           // last, the offered face values (4n)
    double* phi_out;       // [K][n^2] phi^{n+1}
    const double* aN;      // [2][K][n^2] nodal velocity
    const double* aM;      // [2][K][n^2] tensor Chebyshev coefficients
    const double* divN;    // [K][n^2] nodal divergence
    const double* divM;    // [K][n^2] its coefficients
    const double* vface;   // [K][4n] face normal velocity at the element's edge points
    const double* tab;
    const double* gnow;    // ghost row at t^n, or any valid address
    const double* gnext;   // ghost row at t^{n+1}
    int32_t* flag_part;    // [2][nblk]
    double* stat_part;     // [nblk][kStatSlots]
    int nblk, vdeg, rstride;
    // periodic: mask of periodic_mask() (bit 0 x, bit 1 y)
    int kx, ky, K, periodic, cons, cmask, mode, refine, precision, targets, vol, emaxit;
    int iface;             // SL_IFACE_*: edge values by interpolation or backtracking
    double dx, dy, invdx, invdy, dt, vzero, etol;
    double sumW;           // sum of the element's quadrature weights dx dy w_i w_j
    RKTab rk;
    int bs;                // advect block shape: 0 = 256 lanes, 1 = fewest whole waves, 2 = 512 lanes
    // mixed-order meshes (elements grouped in buckets of one order; this
    // launch covers one bucket, K above is its element count)
    const int32_t* elems;  // [K] global element index of the bucket's elements
    const int32_t* nbr;    // [K][MixFace::kPer] face partners of the bucket's elements
    const int32_t* mix;    // device meta data, see MixMeta
    const double* rec_all; // records of all buckets
    const double* interp;  // interpolation matrices between the orders
    int bucket;            // this launch's bucket
};

// Layout of the int32 meta data of a mixed-order mesh on the device:
//   [0, K)               bucket of each global element
//   [K, 2K)              index of each global element within its bucket
//   [2K + kN + b]        nodes per direction of bucket b (b < kMaxBuckets)
//   [2K + kRec + b]      offset of bucket b's records in rec_all (doubles)
//   [2K + kVel + b]      offset of bucket b's nodal velocity in aN_all
//   [2K + kTab + b]      offset of bucket b's tables in tab_all
//   [2K + kK + b]        number of elements of bucket b
//   [2K + kInterp + 16 b_to + b_from]  offset in interp of the n_to x n_from
//                        matrix taking values at b_from's nodes to b_to's
// Bucket b's velocity slice is [2][K_b][n_b^2] (u, then v).
struct MixMeta {
    static constexpr int kN = 0, kRec = kMaxBuckets, kVel = 2 * kMaxBuckets, kTab = 3 * kMaxBuckets,
                         kK = 4 * kMaxBuckets, kInterp = 5 * kMaxBuckets;
    static constexpr int size(int K) { return 2 * K + 5 * kMaxBuckets + kMaxBuckets * kMaxBuckets; }
};

// Face partner table of a mixed-order mesh (int32, bucket order): for element
// position p and side s (left, right, bottom, top), at [p][s][field]: the
// offset in the records of all buckets of the neighbour's trace row on the
// shared face, the neighbour's nodes per direction, and the offset in the
// interpolation matrices of the one from its order to the element's (-1 when
// the orders agree).  Built on the host with the mesh.
struct MixFace {
    static constexpr int kRecOff = 0, kOrder = 1, kInterpOff = 2, kField = 3, kPer = 4 * kField;
};

// face normal velocity of one bucket's elements (aN_all, tab_all: all
// buckets' velocity and tables, located through mix)
int launch_facevel2d_mixed(int n, int K_b, int bucket, int kx, int ky, const int32_t* elems, const int32_t* mix,
                           const double* aN_all, const double* tab_all, const double* interp, double vzero,
                           double* vface, hipStream_t s);
int launch_constrain2d_mixed(int n, const Step2DArgs& A, hipStream_t s);
int advect2d_shapes(int n);            // number of block shapes the advect kernel offers for n
int advect2d_elems(int n, int bs);     // elements per block of shape bs

int launch_prep2d(int n, int K, int has_div, int cons, const double* aN, double* aM, double* divN, double* divM,
                  const double* tab, double dx, double dy, double vscale, int* vdeg, hipStream_t s);
int launch_facevel2d(int n, int kx, int ky, int periodic, const double* aN, const double* tab, double vzero,
                     double* vface, hipStream_t s);
int launch_advect2d(int n, const Step2DArgs& A, hipStream_t s);
int launch_constrain2d(int n, const Step2DArgs& A, hipStream_t s);
// backtracking interface values into the record's last 4n slots (A.phi is phi^n)
int launch_backtrace2d(int n, const Step2DArgs& A, hipStream_t s);
// the advect's mass and energy targets at the upwind edge points (the stage
// sums of the backtraced values about the element's mean), a launch before
// the advect kernel with targets
int launch_targets2d(int n, const Step2DArgs& A, hipStream_t s);
int blocks2d(int n, int K);

// Batched 2D steps (boundary rows, interpolated face values, n >= 4): as
// the 1D ones; the members share n, precision and advect block shape.
// The constrain runs one block per chunk of constrain2d_chunks.
int advect2d_blocks(int n, int bs, int K);
int constrain2d_chunks(int n, int K);
int launch_advect2d_batch(int n, const Step2DArgs& A0, const Step2DArgs* As, const int* start, int nreq,
                          int nblocks, hipStream_t s);
int launch_constrain2d_batch(int n, const Step2DArgs* As, const int* start, int nreq, int nblocks, hipStream_t s);

// One step of a uniform mesh as launch arguments, for launches that step
// several meshes at once (the request loop's batches).  step_prepare
// validates as sl_step (nothing changes on error) and fills L: variant < 0
// if this step cannot join a batch (mixed-order mesh, profiling, 2D target
// or backtracking rows, 2D below four nodes per direction); otherwise the
// arguments of the step from the mesh's current field, its advect variant
// and the block counts of both kernels.  step_commit records the launched
// step on the mesh (field, time, ghost row).
struct StepLaunch {
    int dim, n;
    int variant;  // 1D: advect1d_variant; 2D: precision * 4 + advect block shape
    int adv_blocks, con_blocks;
    Step1DArgs a1;
    Step2DArgs a2;
};
sl_status step_prepare(sl_mesh* m, double dt, const sl_step_opts& opt, StepLaunch* L);
void step_commit(sl_mesh* m, double dt);
// sl_read without waiting on the mesh's stream: for a caller that has seen
// the mesh's last step complete (the stream may hold other meshes' work)
sl_status read_settled(sl_mesh* m, double* u_out, sl_stats* st);
// sl_read without waiting on the mesh's stream: for a caller that has seen
// the mesh's last step complete (the stream may hold other meshes' work)
sl_status read_settled(sl_mesh* m, double* u_out, sl_stats* st);

// 2D boundary tables (4n x 4n, row-major): Qhard = (C_B C_B^T)^+,
// Qsoft = (I + C_B C_B^T)^{-1}; and the reference mass row w (x) w (n^2)
// projected by I - C_B^T Q C_B for each: Zhard, Zsoft
bool build_boundary_tables(const Tables& T, double* Qhard, double* Qsoft, double* Zhard, double* Zsoft);

}  // namespace sl
