// Setup kernels: per-triangle material flags, the fine-level sigma-mass stencil and
// load vector, and the coarse-level mass stencils of the multigrid hierarchy.
//
// Sec. 4 ("Test problem", "Simulation setup"): P1 elements on the triangulation,
// sigma and the current density piecewise constant per region. The consistent P1
// mass of a triangle is sigma |T|/12 [[2,1,1],[1,2,1],[1,1,2]] and the exact load of
// a constant density J is J |T|/3 per vertex. On the uniform SW-NE split grid every
// triangle has |T| = h^2/2.
#include "pt_device.h"

namespace pt {

struct SetupArgs {
    int n, side;
    double h;
    pt_rect sig, nu, coil;
    double sigma_in, J0;
    const double* d_sigma;  // optional per-triangle conductivity
    const uint8_t* region;  // region mode: [2 n^2] region of every triangle (null: rectangles)
    const double* rsj;      // region mode: [kMaxRegions][2] conductivity and current amplitude
    uint8_t* flags;         // [2 n^2] region of every triangle (rectangles: 1 inside nu_rect, else 0)
    double* sig_out;        // [2 n^2] per-triangle conductivity (written if non-null)
    double* mt;             // [4][nodes] fine mass stencil
    double* b;              // [nodes] load amplitude
};

__device__ __forceinline__ bool in_rect(const pt_rect& r, double x, double y) {
    return x >= r.x0 && x <= r.x1 && y >= r.y0 && y <= r.y1;
}

// Centroid of triangle (i, j, t): t = 0 -> ((3i+2)/(3n), (3j+1)/(3n)), t = 1 -> ((3i+1)/(3n), (3j+2)/(3n)).
__device__ __forceinline__ void centroid(int n, int i, int j, int t, double& cx, double& cy) {
    double d = 3.0 * (double)n;
    cx = (double)(3 * i + (t == 0 ? 2 : 1)) / d;
    cy = (double)(3 * j + (t == 0 ? 1 : 2)) / d;
}

__device__ __forceinline__ double tri_sigma(const SetupArgs& a, int i, int j, int t) {
    if (i < 0 || j < 0 || i >= a.n || j >= a.n) return 0.0;
    if (a.region) return a.rsj[2 * a.region[2 * (j * a.n + i) + t]];
    if (a.d_sigma) return a.d_sigma[2 * (j * a.n + i) + t];
    double cx, cy;
    centroid(a.n, i, j, t, cx, cy);
    return in_rect(a.sig, cx, cy) ? a.sigma_in : 0.0;
}

__device__ __forceinline__ double tri_J(const SetupArgs& a, int i, int j, int t) {
    if (i < 0 || j < 0 || i >= a.n || j >= a.n) return 0.0;
    if (a.region) return a.rsj[2 * a.region[2 * (j * a.n + i) + t] + 1];
    double cx, cy;
    centroid(a.n, i, j, t, cx, cy);
    return in_rect(a.coil, cx, cy) ? a.J0 : 0.0;
}

__global__ void __launch_bounds__(kBlock) k_tri_flags(SetupArgs a) {
    size_t ntri = 2 * (size_t)a.n * a.n;
    for (size_t t = blockIdx.x * (size_t)kBlock + threadIdx.x; t < ntri; t += (size_t)gridDim.x * kBlock) {
        int typ = (int)(t & 1);
        size_t c = t >> 1;
        int i = (int)(c % a.n), j = (int)(c / a.n);
        double cx, cy;
        centroid(a.n, i, j, typ, cx, cy);
        a.flags[t] = a.region ? a.region[t] : (in_rect(a.nu, cx, cy) ? 1 : 0);
        if (a.sig_out) a.sig_out[t] = tri_sigma(a, i, j, typ);
    }
}

// Node (i, j) touches T_a(i,j), T_b(i,j), T_a(i-1,j), T_b(i,j-1), T_a(i-1,j-1), T_b(i-1,j-1).
// Edge couplings: east (i,j)-(i+1,j) lies in T_a(i,j) and T_b(i,j-1); north (i,j)-(i,j+1)
// in T_b(i,j) and T_a(i-1,j); north-east (i,j)-(i+1,j+1) in T_a(i,j) and T_b(i,j).
__global__ void __launch_bounds__(kBlock) k_fine_node(SetupArgs a) {
    size_t nodes = (size_t)a.side * a.side;
    double area = 0.5 * a.h * a.h;
    for (size_t id = blockIdx.x * (size_t)kBlock + threadIdx.x; id < nodes; id += (size_t)gridDim.x * kBlock) {
        int i = (int)(id % a.side), j = (int)(id / a.side);
        double s_aij = tri_sigma(a, i, j, 0), s_bij = tri_sigma(a, i, j, 1);
        double s_a_w = tri_sigma(a, i - 1, j, 0), s_b_s = tri_sigma(a, i, j - 1, 1);
        double s_a_sw = tri_sigma(a, i - 1, j - 1, 0), s_b_sw = tri_sigma(a, i - 1, j - 1, 1);
        double ssum = s_aij + s_bij + s_a_w + s_b_s + s_a_sw + s_b_sw;
        a.mt[id] = ssum * area / 6.0;
        a.mt[nodes + id] = (s_aij + s_b_s) * area / 12.0;
        a.mt[2 * nodes + id] = (s_bij + s_a_w) * area / 12.0;
        a.mt[3 * nodes + id] = (s_aij + s_bij) * area / 12.0;
        double jsum = tri_J(a, i, j, 0) + tri_J(a, i, j, 1) + tri_J(a, i - 1, j, 0) + tri_J(a, i, j - 1, 1) +
                      tri_J(a, i - 1, j - 1, 0) + tri_J(a, i - 1, j - 1, 1);
        bool interior = i > 0 && j > 0 && i < a.n && j < a.n;
        a.b[id] = interior ? jsum * area / 3.0 : 0.0;
    }
}

// Weight of coarse node J in the P1 interpolation at fine node (fi, fj): the offset
// o = (fi, fj) - 2 J must be (0,0) -> 1 or one of (+-1,0), (0,+-1), (1,1), (-1,-1) -> 1/2.
__device__ __forceinline__ double pweight(int fi, int fj, int ci, int cj) {
    int ox = fi - 2 * ci, oy = fj - 2 * cj;
    if (ox == 0 && oy == 0) return 1.0;
    if ((ox == 1 || ox == -1) && oy == 0) return 0.5;
    if ((oy == 1 || oy == -1) && ox == 0) return 0.5;
    if ((ox == 1 && oy == 1) || (ox == -1 && oy == -1)) return 0.5;
    return 0.0;
}

// Galerkin coarse mass M_c = P^T M_f P with P the P1 interpolation of the nested
// SW-NE grids: M_c[I, J] = sum_a P[a, I] sum_b M_f[a, b] P[b, J] over the fine
// support of I and the 7-point neighbourhood of a (the same for a Khat table). Boundary
// nodes get the centre value bdiag and no couplings: 0 for the mass; 1 for Khat, whose
// diagonal divides in the Jacobi step (the vector entries there are zero, so they stay zero).
__global__ void __launch_bounds__(kBlock) k_galerkin(const double* mf, int sf, double* mc, int sc, double bdiag) {
    size_t nf = (size_t)sf * sf, ncn = (size_t)sc * sc;
    const int oxs[7] = {0, 1, -1, 0, 0, 1, -1};
    const int oys[7] = {0, 0, 0, 1, -1, 1, -1};
    for (size_t id = blockIdx.x * (size_t)kBlock + threadIdx.x; id < ncn; id += (size_t)gridDim.x * kBlock) {
        int ci = (int)(id % sc), cj = (int)(id / sc);
        double out[4] = {0, 0, 0, 0};
        bool interior = ci > 0 && cj > 0 && ci < sc - 1 && cj < sc - 1;
        if (interior) {
            const int jx[4] = {ci, ci + 1, ci, ci + 1};
            const int jy[4] = {cj, cj, cj + 1, cj + 1};
            for (int ia = 0; ia < 7; ++ia) {
                int ai = 2 * ci + oxs[ia], aj = 2 * cj + oys[ia];
                double wa = (ia == 0) ? 1.0 : 0.5;
                size_t a = (size_t)aj * sf + ai;
                // row a of M_f: (b, value)
                double mv[7];
                int bi[7], bj[7];
                mv[0] = mf[a];
                bi[0] = ai; bj[0] = aj;
                mv[1] = mf[nf + a];                 bi[1] = ai + 1; bj[1] = aj;
                mv[2] = mf[nf + a - 1];             bi[2] = ai - 1; bj[2] = aj;
                mv[3] = mf[2 * nf + a];             bi[3] = ai;     bj[3] = aj + 1;
                mv[4] = mf[2 * nf + a - sf];        bi[4] = ai;     bj[4] = aj - 1;
                mv[5] = mf[3 * nf + a];             bi[5] = ai + 1; bj[5] = aj + 1;
                mv[6] = mf[3 * nf + a - sf - 1];    bi[6] = ai - 1; bj[6] = aj - 1;
                for (int ib = 0; ib < 7; ++ib) {
                    double v = wa * mv[ib];
                    if (v == 0.0) continue;
                    for (int q = 0; q < 4; ++q) out[q] += v * pweight(bi[ib], bj[ib], jx[q], jy[q]);
                }
            }
        }
        mc[id] = interior ? out[0] : bdiag;
        mc[ncn + id] = out[1];
        mc[2 * ncn + id] = out[2];
        mc[3 * ncn + id] = out[3];
    }
}

static int grid_for(size_t items) {
    size_t g = (items + kBlock - 1) / kBlock;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

void launch_setup_fine(const Plan& p, char* ws, hipStream_t st) {
    // one pass per batch instance: the iron flags and the load are the instance's own, the
    // mass stencil (shared conductivity) is the same for all and rewritten each time
    for (int inst = 0; inst < p.B; ++inst) {
        const pt_problem& q = p.probs[inst];
        SetupArgs a;
        a.n = p.n;
        a.side = p.side;
        a.h = p.h;
        a.sig = q.sigma_rect;
        a.nu = q.nu_rect;
        a.coil = q.coil_rect;
        a.sigma_in = q.sigma_in;
        a.J0 = q.J0;
        a.d_sigma = q.d_sigma;
        a.region = p.region_mode ? q.d_region : nullptr;
        a.rsj = (const double*)(ws + p.off_rsj);
        a.flags = (uint8_t*)(ws + p.off_flags) + (size_t)inst * 2 * p.n * p.n;
        a.mt = (double*)(ws + p.lev[0].off_mt);
        a.b = (double*)(ws + p.off_b) + (size_t)inst * p.nodes;
        a.sig_out = (p.opt.adjoint && inst == 0) ? (double*)(ws + p.off_sig) : nullptr;
        hipLaunchKernelGGL(k_tri_flags, dim3(grid_for(2 * (size_t)p.n * p.n)), dim3(kBlock), 0, st, a);
        hipLaunchKernelGGL(k_fine_node, dim3(grid_for(p.nodes)), dim3(kBlock), 0, st, a);
    }
}

void launch_galerkin_table(const Plan& p, char* ws, int l, bool khat, hipStream_t st) {
    const LevelDesc& f = p.lev[l];
    const LevelDesc& c = p.lev[l + 1];
    const size_t fo = khat ? f.off_kt : f.off_mt, co = khat ? c.off_kt : c.off_mt;
    hipLaunchKernelGGL(k_galerkin, dim3(grid_for(c.nodes)), dim3(kBlock), 0, st, (const double*)(ws + fo), f.side,
                       (double*)(ws + co), c.side, khat ? 1.0 : 0.0);
}

void launch_galerkin(const Plan& p, char* ws, int l, hipStream_t st) { launch_galerkin_table(p, ws, l, false, st); }

// Khat = S_nuhat, the P1 stiffness with the per-triangle coefficient nu_hat of the triangle's
// region, as a stencil table in the mass layout (centre, E, N, NE per node). On the SW-NE split
// grid the P1 coupling of two nodes through a triangle is -nuhat_T cot(theta) / 2 with theta the
// angle opposite their edge: 45 degrees for the axis edges (each in two triangles, one on either
// side), 90 degrees for the diagonal ones (no coupling). So the east weight of node (i, j) is
// (nuhat(T_a(i,j)) + nuhat(T_b(i,j-1))) / 2, the north weight (nuhat(T_b(i,j)) + nuhat(T_a(i-1,j))) / 2,
// and the centre the sum of the four axis weights (a constant nu_hat gives 4 nu, -nu, -nu, 0).
struct StiffArgs {
    int n, side;
    const uint8_t* region;  // [2 n^2]
    const double* rkh;      // [kMaxRegions] nu_hat of each region
    double* kt;             // [4][nodes]
};

__device__ __forceinline__ double tri_khat(const StiffArgs& a, int i, int j, int t) {
    if (i < 0 || j < 0 || i >= a.n || j >= a.n) return 0.0;
    return a.rkh[a.region[2 * (j * a.n + i) + t]];
}

__global__ void __launch_bounds__(kBlock) k_fine_stiffness(StiffArgs a) {
    const size_t nodes = (size_t)a.side * a.side;
    for (size_t id = blockIdx.x * (size_t)kBlock + threadIdx.x; id < nodes; id += (size_t)gridDim.x * kBlock) {
        const int i = (int)(id % a.side), j = (int)(id / a.side);
        const double we = 0.5 * (tri_khat(a, i, j, 0) + tri_khat(a, i, j - 1, 1));
        const double ww = 0.5 * (tri_khat(a, i - 1, j, 0) + tri_khat(a, i - 1, j - 1, 1));
        const double wn = 0.5 * (tri_khat(a, i, j, 1) + tri_khat(a, i - 1, j, 0));
        const double ws = 0.5 * (tri_khat(a, i, j - 1, 1) + tri_khat(a, i - 1, j - 1, 0));
        const bool interior = i > 0 && j > 0 && i < a.n && j < a.n;
        a.kt[id] = interior ? we + ww + wn + ws : 1.0;   // (boundary: as in k_galerkin)
        a.kt[nodes + id] = -we;
        a.kt[2 * nodes + id] = -wn;
        a.kt[3 * nodes + id] = 0.0;
    }
}

void launch_setup_stiffness(const Plan& p, char* ws, hipStream_t st) {
    StiffArgs a;
    a.n = p.n;
    a.side = p.side;
    a.region = p.prob.d_region;
    a.rkh = (const double*)(ws + p.off_rkh);
    a.kt = (double*)(ws + p.lev[0].off_kt);
    hipLaunchKernelGGL(k_fine_stiffness, dim3(grid_for(p.nodes)), dim3(kBlock), 0, st, a);
}

}  // namespace pt
