// Internal declarations shared by the kernel translation units and the C ABI layer.
//
// Working layouts in the workspace (all node-major, so that the time axis and the
// frequency axis are contiguous for every node):
//   time series    double [nodes][N]        (Uw, Fw: iterate and explicit load)
//   slot vectors   T2     [nodes][S], S=N/2 (T2 = double2 in FP64 mode, float2 in
//                                            FP32 mode); slot 0 carries the two real
//                                            systems k = 0 (.x) and k = N/2 (.y)
//   M stencil      double [4][nodes] per multigrid level: centre, east (i,i+1),
//                  north (i,i+side), north-east (i,i+side+1) couplings of the
//                  sigma-weighted mass (symmetric, so west/south/south-west come
//                  from the neighbour's entries)
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "ptsolve.h"

namespace pt {

constexpr int kBlock = 256;          // threads per workgroup in every kernel
constexpr int kMaxLevels = 16;
constexpr int kNumXcd = 8;
constexpr int kReduceRows = 64;      // first-stage row groups of the dot-product reduction
constexpr int kReduceBatch = 8;      // partials whose loads a reduction thread issues together
constexpr int kAdjBlocks = 8192;     // workgroups of the grid-stride adjoint kernels
constexpr int kCocgRows = 4096;      // workgroups along the nodes of the COCG vector kernels, at most
constexpr int kRecDoubles = 16;      // residual-sweep record per node: mass row, load, reluctivity laws
constexpr int kRecDoublesExp = 24;   // the same with the exp-capped law (four parameters per triangle)
constexpr int kMaxRegions = 16;      // material regions of a problem (the triangles' region ids)

// Per-slot scalar in "generic" form: for slot s >= 1 a complex number (x + i y);
// for slot 0 two reals, x acting on the real part (k = 0) and y on the imaginary
// part (k = N/2). Applying it to a slot value w is
//   (a w.x - b w.y,  c w.y + b w.x)
// with (a, b, c) = (x, y, x) for s >= 1 and (x, 0, y) for s = 0.

struct LevelDesc {
    int n;          // cells per side at this level
    int side;       // n + 1
    size_t nodes;   // side * side
    size_t off_mt;  // M stencil table, 4 * nodes doubles
    size_t off_kt;  // Khat stencil table in the same layout (per-region Khat only, else 0)
    size_t off_r;   // slot vector: right-hand side at this level
    size_t off_x;   // slot vector: correction at this level
};

// Launch geometry of the node-sweeping kernels. A workgroup owns per_step adjacent grid
// columns and walks down one chunk of rows_per_chunk rows, one row per loop step, so
// the stencil neighbours in the rows above and below are the rows it has just touched
// (and that the workgroups of the adjacent columns, scheduled on the same XCD at the
// same time, are touching). Workgroup vb -> column group vb % col_groups, row chunk
// vb / col_groups.
struct Geom {
    int per_step;        // columns (nodes per row step) per workgroup
    int slot_chunk;      // slots per workgroup (slot-vector kernels) or team size (time kernels)
    int chunks;          // workgroups along y (slot chunks)
    int col_groups;      // ceil(side / per_step)
    int rows_per_chunk;  // rows per workgroup
    int blocks;          // workgroups along x (multiple of kNumXcd)
};

// Kernel classes of the per-launch event timer (order matches pt_kernel_class_name).
enum KernelId {
    KID_SETUP = 0,
    KID_TRANSPOSE,
    KID_RESIDUAL,     // residual sweep F - A(U)
    KID_RFFT,         // packed real DFT along time
    KID_REDUCE,       // norm and dot-product reductions, per-slot scalar kernels
    KID_DOWN0,        // V-cycle restriction from the finest level
    KID_DOWNC,        // V-cycle restriction on coarser levels
    KID_COARSEST,
    KID_UP0,          // V-cycle prolongation + smoothing onto the finest level
    KID_UPC,
    KID_MATVEC,       // (Khat + z M) p with fused dot products
    KID_INVERSE,      // inverse DFT + iterate update
    KID_COCG,         // COCG vector updates and copies
    KID_MEMSET,
    KID_OTHER,
    KID_COUNT
};

struct Timer {
    static constexpr int kCap = 256;
    bool on = false;
    unsigned mask = ~0u;   // kernel classes that are timed (bit per class)
    int used = 0;
    hipEvent_t ev[2 * kCap];
    int kid[kCap];
    double ms[KID_COUNT];
    long long cnt[KID_COUNT];
};

void tm_begin(const struct Plan& p, int kid, hipStream_t st);
void tm_end(const struct Plan& p, int kid, hipStream_t st);

struct Plan {
    pt_problem prob;     // instance 0 (the shared grid, period, conductivity and nu_max)
    pt_options opt;
    int B;               // instances in the batch (power of two; 1 for a single problem)
    pt_problem* probs;   // host copy of the B instances
    int n, N, S, side;
    int ST;              // slots (and time pairs) per node over all instances: B S
    size_t nodes;
    bool fp32;
    size_t elem;        // bytes per slot value (16 or 8)
    double tau, h;
    int nlev;
    LevelDesc lev[kMaxLevels];
    // workspace offsets (bytes)
    size_t off_U, off_F, off_P, off_cx, off_cr, off_cq, off_cp;
    size_t off_flags, off_b, off_tw64, off_tw32, off_zs, off_wave;
    size_t off_rec;     // per-instance, per-node records of the residual sweep (rec_doubles(law) doubles)
    size_t off_npart, off_caux;  // COCG plans: r^H r partials, per-slot scalars and counter
    int inner_done;              // inner steps of the last inner solve
    int inner_max;               // most inner steps of one outer step in the current call
    long long inner_sum;         // inner steps over the current call
    size_t off_part, part_bytes, off_scal, off_flag, off_coef, off_coef2, off_hist, off_inst;
    size_t off_L, off_G, off_sig;   // adjoint plans: adjoint iterate, dl/dU, per-triangle sigma
    size_t off_R, off_Ut, off_D, off_V, off_Z;  // Newton plans: residual, trial, step, Krylov bases
    size_t tf_stride;                           // bytes between consecutive Krylov basis fields
    size_t ws_bytes;
    bool has_cocg_vectors;
    bool vc_pre;        // the cycle pre-smooths (V(1,1)); otherwise V(0,1)
    // host copies of the small tables uploaded at every call
    double* h_tw64;     // N complex: exp(-2 pi i k / N)
    float* h_tw32;      // N complex, float
    double* h_zs;       // ST x 3: generic (a, b, c) of the shift z_s, repeated per instance
    double* h_wave;     // B x N: w(2 pi t_{j+1} / T) of each instance
    double* h_inst;     // B x 4: nu_a, nu_b, nu_out, 0 of each instance
    int law;            // pt_nu_law of every region
    int nreg;           // regions (2 in rectangle mode: 0 outside, 1 the nu rectangle)
    bool region_mode;   // materials from d_region and the region table
    pt_region regions[kMaxRegions];  // region mode: host copy of the regions
    double* h_regp;     // B x kMaxRegions x 4: law parameters of each region (see law_nu)
    double* h_rsj;      // kMaxRegions x 2: conductivity and current amplitude (region mode)
    double h_rkh[kMaxRegions];  // Khat coefficient of each region (nu_max where nu_hat is 0)
    bool vk;            // Khat = S_nuhat with a per-region coefficient (stencil tables off_kt)
    size_t off_regp, off_rsj, off_rkh;
    int target_slot, target_team;  // grid targets of the slot-vector and per-node kernels
    int target_down, target_up;    // grid targets of the restriction and up sweeps (all levels)
    Geom g_slot0;       // up sweep on level 0 (its dot partials: one row per workgroup)
    Geom g_mv;          // operator apply on level 0: two adjacent columns per team
    Geom g_team;        // per-node team kernels (inverse DFT)
    Geom g_fwd;         // residual sweep (team of min(S, 256) threads per column)
    Timer* tm;          // per-kernel event timer (owned by the plan)
    struct GraphCache* gr;  // captured outer steps (owned by the plan)
};

void graph_release(Plan& p);

// target = number of workgroups (per slot chunk) the sweeping kernels aim for. The
// per-node team kernels sweep B (n+1) virtual columns (instance b, grid column i at
// b (n+1) + i) over n+1 rows.
Geom slot_geom(int side, int S, int V, int target, int cols = 0, int max_chunk = kBlock);
Geom team_geom(int side, int S, int B, int target);
Geom fwd_geom(int side, int S, int B, int target);

// ---------------------------------------------------------------- launchers
// setup (k_setup.hip)
void launch_setup_fine(const Plan& p, char* ws, hipStream_t st);
void launch_galerkin(const Plan& p, char* ws, int l, hipStream_t st);
void launch_galerkin_table(const Plan& p, char* ws, int l, bool khat, hipStream_t st);
void launch_setup_stiffness(const Plan& p, char* ws, hipStream_t st);
void launch_row_records(const Plan& p, char* ws, hipStream_t st);
// time axis (k_time.hip)
void launch_transpose_in(const Plan& p, const double* src, double* dst, hipStream_t st);
void launch_transpose_out(const Plan& p, const double* src, double* dst, hipStream_t st);
enum TimeMode { TM_RESIDUAL = 0, TM_SIGNAL = 1 };
// forward: residual (or the field itself) per node, packed real DFT to slot vector
// out (if non-null), real residual to rout (if non-null), norm partials to part. Returns the
// partial layout for launch_reduce_norms: 0 for the column sweeps' layout, else the number of
// partial pairs of the generic kernel (one per workgroup).
int launch_forward(const Plan& p, char* ws, int mode, const double* Uw, void* out, double* rout,
                   double* part, hipStream_t st);
void launch_reduce_norms(const Plan& p, char* ws, double* part, int flat, double* out2,
                         hipStream_t st);
// packed real DFT of rt (T2 [nodes][ST], solver precision) into out; conj: conjugate the
// result (every slot but the packed real slot 0)
void launch_rfft(const Plan& p, char* ws, const void* rt, void* out, int conj, hipStream_t st);
// inverse: Uw (+)= (1/N) irfft(c(coef (x) xhat)), coef may be null (identity), c the
// conjugation (conj = 1) or the identity
void launch_inverse(const Plan& p, char* ws, const void* xhat, const double* coef, double* Uw,
                    int accumulate, hipStream_t st, int conj = 0);
// sum nparts pairs of partials in a fixed order into out2[0], out2[1]
void launch_reduce_pairs(const Plan& p, const double* part, int nparts, double* out2, hipStream_t st);
// adjoint (k_adjoint.hip)
void launch_adj_source(const Plan& p, char* ws, hipStream_t st);
int launch_adj_residual(const Plan& p, char* ws, void* rt, hipStream_t st);  // returns the partial count
void launch_adj_grad(const Plan& p, char* ws, bool with_lambda, double* gth, double* gsg, int per_cell,
                     hipStream_t st);
// out = J v (b null) or b - J v, J the linearised operator at the state in the iterate buffer;
// dir = +1: J, dir = -1: J^T
void launch_jac_apply(const Plan& p, char* ws, const double* v, const double* b, double* out, int dir,
                      hipStream_t st);
// time-field vector operations (k_krylov.hip); launch_tdot returns the partial count
int launch_tdot(const Plan& p, const double* a, const double* b, double* part, hipStream_t st);
void launch_taxpby(const Plan& p, double alpha, const double* x, double beta, double* y, hipStream_t st);
void launch_apply_K(const Plan& p, char* ws, const double* u, double* ku, int nslices,
                    hipStream_t st);
void launch_reciprocals(const double* x, double* y, long n, hipStream_t st);
// frequency (k_freq.hip)
void launch_vcycle(const Plan& p, char* ws, const void* r0, void* x0, int dotmode, double* part,
                   hipStream_t st);
enum DotMode { DOT_NONE = 0, DOT_HERM = 1, DOT_BILIN = 2 };
// y = A x (optional y), partials of x . (A x) with dotmode
void launch_matvec(const Plan& p, char* ws, const void* x, void* y, int dotmode, double* part,
                   hipStream_t st);
// reduce dot partials -> generic scalars out[S] (double2)
void launch_reduce_dots(const Plan& p, double* part, int nblk, int dotmode, double* out, hipStream_t st);
// num, den = the reductions of the partials pa (na workgroups) and pb (nb workgroups); coef = num / den
void launch_reduce_ratio(const Plan& p, double* pa, int na, double* pb, int nb, int dotmode, double* num, double* den,
                         double* coef, hipStream_t st);
// COCG vector kernels: mode 0 (x += a (x) p, r -= a (x) q) or 1 (r = src), both leaving the
// Hermitian partials of r^H r in part (cocg_rows(p) rows)
void launch_cocg_vec(const Plan& p, int mode, const double* coef, void* x, void* r, const void* src,
                     const void* q, double* part, hipStream_t st);
int cocg_rows(const Plan& p);
// per-slot COCG scalars (double2 arrays of ST entries) and their stage-2 reductions
struct CocgScalars {
    double *nr, *thr, *act, *rho, *coef;
    int *count, *flag;
    double eta2, btol;
};
enum CocgReduceOp { COCG_NORM0 = 0, COCG_NORM = 1, COCG_ALPHA = 2, COCG_RHO = 3, COCG_BETA = 4 };
void launch_cocg_reduce(const Plan& p, double* part, int nblk, int op, const CocgScalars& cs, hipStream_t st);
// p = z + b (x) p
void launch_cocg_p(const Plan& p, const double* coef, const void* z, void* pv, hipStream_t st);
void launch_copy_slots(const Plan& p, const void* src, void* dst, hipStream_t st);
// byte counts are multiples of 16, pointers 16-byte aligned
void launch_copy16(const void* src, void* dst, size_t bytes, hipStream_t st);
void launch_zero16(void* dst, size_t bytes, hipStream_t st);

}  // namespace pt
