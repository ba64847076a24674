// Adjoint kernels: the source dl/dU of the cycle-averaged eddy-current loss, the residual
// of the transposed linearised periodic system, and the parameter gradients.
//
// Loss (the Joule loss of one period with the implicit-Euler difference quotient and the
// consistent sigma-mass): l(U) = tau sum_n (d u^n)^T M (d u^n), d u^n = (u^n - u^{n-1})/tau.
// The state U solves A(U) = F (eqs. (disc1)-(disc2)); J = dA/dU has the diagonal blocks
// M/tau + K'(u^n) and the cyclic sub-diagonal blocks -M/tau, so the adjoint state solves
//   (M/tau)(lambda^n - lambda^{n+1}) + K'(u^n) lambda^n = g^n,  lambda^{N+1} = lambda^1,
// with g^n = dl/du^n = (2/tau) M (2 u^n - u^{n-1} - u^{n+1}): backward in time, periodic.
// K'(u) is symmetric (K is the gradient of an energy); per triangle it is
//   |T| grad phi_a . (nu I + 2 dnu/d(s^2) grad u grad u^T) grad phi_b,
// with the law of the triangle's region (law_nu_dn; dnu/d(s^2) the right derivative at the kink
// of the exp-capped law).
//
// Layout as everywhere on the time axis: node-major [nodes][N] doubles, boundary nodes 0.
// Scaled gradients G = h grad (differences of nodal values) as in the forward sweep, so
// that |T| grad v . grad w = G_v . G_w / 2 on the uniform grid.
#include "pt_device.h"

namespace pt {

struct AdjArgs {
    int n, side, N, lgN;
    size_t nodes;
    double tau, inv_tau, n2;
    const double4* regp;   // [kMaxRegions] law parameters of each region (law_nu)
    const double* U;       // primal solution [nodes][N]
    const double* L;       // adjoint iterate [nodes][N]
    const double* G;       // dl/dU [nodes][N]
    const double* mt;      // fine mass stencil [4][nodes]
    const uint8_t* flags;  // [2 n^2] region of every triangle
    const double* theta;   // [2 n^2] or null
    const double* sig;     // [2 n^2] per-triangle conductivity
    double* part;          // norm / loss partials, two per workgroup
};

// nu and 2 n^2 dnu/d(s^2) of one triangle from the scaled gradient of u.
struct Law {
    double nu, dn;
};

template <int LAW>
__device__ __forceinline__ Law tri_law_q(const double4 q, double n2, double th, double gx, double gy) {
    Law L;
    const double s2 = n2 * (gx * gx + gy * gy);
    double dn;
    L.nu = th * law_nu_dn<LAW>(q, s2, dn);
    L.dn = 2.0 * n2 * th * dn;
    return L;
}
template <int LAW>
__device__ __forceinline__ Law tri_law(const AdjArgs& a, int region, double th, double gx, double gy) {
    return tri_law_q<LAW>(a.regp[region], a.n2, th, gx, gy);
}

// Per-triangle tables at an index that is the same on every lane when UNI (read through the
// scalar unit; the region byte from the aligned word that holds it: the table has 2 n^2 bytes,
// a multiple of 4).
template <bool UNI>
__device__ __forceinline__ int region_of(const AdjArgs& a, size_t tri) {
    if constexpr (UNI) {
        const uint32_t w = uload<true>((const uint32_t*)a.flags, tri >> 2);
        return (int)((w >> (8 * (tri & 3))) & 0xffu);
    } else {
        return a.flags[tri];
    }
}

// Contribution of one triangle to (K'(u) lambda)_i / 1: half of
// nu G_l . dphi + dn (G_u . G_l)(G_u . dphi), dphi the scaled gradient of phi_i.
__device__ __forceinline__ double tri_lin(const Law& L, double ux, double uy, double lx, double ly, int px, int py) {
    const double ul = ux * lx + uy * ly;
    const double lp = lx * px + ly * py;
    const double up = ux * px + uy * py;
    return 0.5 * (L.nu * lp + L.dn * ul * up);
}

struct Stencil {
    double c, e, w, nn, s, ne, sw;
};

__device__ __forceinline__ Stencil load_stencil(const double* X, size_t node, size_t sd, int N, int t) {
    Stencil v;
    const size_t NN = (size_t)N;
    v.c = X[node * NN + t];
    v.e = X[(node + 1) * NN + t];
    v.w = X[(node - 1) * NN + t];
    v.nn = X[(node + sd) * NN + t];
    v.s = X[(node - sd) * NN + t];
    v.ne = X[(node + sd + 1) * NN + t];
    v.sw = X[(node - sd - 1) * NN + t];
    return v;
}

struct MassRow {
    double c, e, w, nn, s, ne, sw;
    bool any;
};

template <bool UNI = false>
__device__ __forceinline__ MassRow mass_row(const AdjArgs& a, size_t node) {
    const size_t nd = a.nodes, sd = a.side;
    MassRow m;
    m.c = uload<UNI>(a.mt, node);
    m.e = uload<UNI>(a.mt, nd + node);
    m.w = uload<UNI>(a.mt, nd + node - 1);
    m.nn = uload<UNI>(a.mt, 2 * nd + node);
    m.s = uload<UNI>(a.mt, 2 * nd + node - sd);
    m.ne = uload<UNI>(a.mt, 3 * nd + node);
    m.sw = uload<UNI>(a.mt, 3 * nd + node - sd - 1);
    m.any = (m.c != 0.0) || (m.e != 0.0) || (m.w != 0.0) || (m.nn != 0.0) || (m.s != 0.0) || (m.ne != 0.0) ||
            (m.sw != 0.0);
    return m;
}

__device__ __forceinline__ double mass_apply(const MassRow& m, const Stencil& v) {
    return m.c * v.c + m.e * v.e + m.w * v.w + m.nn * v.nn + m.s * v.s + m.ne * v.ne + m.sw * v.sw;
}

__device__ __forceinline__ void block_pair_sum(double x, double y, double* out) {
    __shared__ double red[2][kBlock];
    red[0][threadIdx.x] = x;
    red[1][threadIdx.x] = y;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = red[0][0];
        out[1] = red[1][0];
    }
}

// g^n = (2/tau) M (2 u^n - u^{n-1} - u^{n+1}) at interior nodes, 0 elsewhere.
__global__ void __launch_bounds__(kBlock) k_adj_source(AdjArgs a, double* g) {
    const size_t total = a.nodes * (size_t)a.N;
    const size_t sd = a.side;
    for (size_t id = (size_t)virtual_block_of(blockIdx.x, gridDim.x, 1) * kBlock + threadIdx.x; id < total;
         id += (size_t)gridDim.x * kBlock) {
        const size_t node = id >> a.lgN;
        const int t = (int)(id & (size_t)(a.N - 1));
        const int i = (int)(node % sd), j = (int)(node / sd);
        double out = 0.0;
        if (i > 0 && j > 0 && i < a.n && j < a.n) {
            const MassRow m = mass_row(a, node);
            if (m.any) {
                const int tp = t == 0 ? a.N - 1 : t - 1, tn = t + 1 == a.N ? 0 : t + 1;
                const Stencil u0 = load_stencil(a.U, node, sd, a.N, t);
                const Stencil um = load_stencil(a.U, node, sd, a.N, tp);
                const Stencil up = load_stencil(a.U, node, sd, a.N, tn);
                out = 2.0 * a.inv_tau * (2.0 * mass_apply(m, u0) - mass_apply(m, um) - mass_apply(m, up));
            }
        }
        g[id] = out;
    }
}

// R^n = g^n - (M/tau)(lambda^n - lambda^{n+1}) - K'(u^n) lambda^n at interior nodes (0 on the
// boundary), written in the solver precision T for the time DFT; norm partials of R and g.
// UNI (N >= 64): the 64 lanes of a wavefront hold 64 consecutive time levels of one node (every
// wavefront starts at a multiple of 64 and N is a multiple of 64), so the node's tables are read
// through the scalar unit.
template <typename T, int LAW, bool UNI>
__global__ void __launch_bounds__(kBlock) k_adj_residual(AdjArgs a, T* rt) {
    const size_t total = a.nodes * (size_t)a.N;
    const size_t sd = a.side;
    double rr = 0.0, gg = 0.0;
    for (size_t id = (size_t)virtual_block_of(blockIdx.x, gridDim.x, 1) * kBlock + threadIdx.x; id < total;
         id += (size_t)gridDim.x * kBlock) {
        size_t node = id >> a.lgN;
        if constexpr (UNI) node = (size_t)__builtin_amdgcn_readfirstlane((int)node);
        const int t = (int)(id & (size_t)(a.N - 1));
        const int i = (int)(node % sd), j = (int)(node / sd);
        double R = 0.0;
        if (i > 0 && j > 0 && i < a.n && j < a.n) {
            const double g = a.G[id];
            const Stencil u = load_stencil(a.U, node, sd, a.N, t);
            const Stencil l = load_stencil(a.L, node, sd, a.N, t);
            const size_t c_ij = (size_t)j * a.n + i, c_w = c_ij - 1, c_s = c_ij - a.n, c_sw = c_ij - a.n - 1;
            const size_t tri[6] = {2 * c_ij, 2 * c_ij + 1, 2 * c_w, 2 * c_s + 1, 2 * c_sw, 2 * c_sw + 1};
            // scaled gradients of u and lambda on the six triangles and the node's dphi
            const double gux[6] = {u.e - u.c, u.ne - u.nn, u.c - u.w, u.e - u.c, u.s - u.sw, u.c - u.w};
            const double guy[6] = {u.ne - u.e, u.nn - u.c, u.nn - u.c, u.c - u.s, u.c - u.s, u.w - u.sw};
            const double glx[6] = {l.e - l.c, l.ne - l.nn, l.c - l.w, l.e - l.c, l.s - l.sw, l.c - l.w};
            const double gly[6] = {l.ne - l.e, l.nn - l.c, l.nn - l.c, l.c - l.s, l.c - l.s, l.w - l.sw};
            const int px[6] = {-1, 0, 1, -1, 0, 1};
            const int py[6] = {0, -1, -1, 1, 1, 0};
            double Kl = 0.0;
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                const double th = a.theta ? uload<UNI>(a.theta, tri[k]) : 1.0;
                const size_t rq = 4 * (size_t)region_of<UNI>(a, tri[k]);
                const double* rp = (const double*)a.regp;
                const double4 q = make_double4(uload<UNI>(rp, rq), uload<UNI>(rp, rq + 1), uload<UNI>(rp, rq + 2),
                                               uload<UNI>(rp, rq + 3));
                const Law L = tri_law_q<LAW>(q, a.n2, th, gux[k], guy[k]);
                Kl += tri_lin(L, gux[k], guy[k], glx[k], gly[k], px[k], py[k]);
            }
            R = g - Kl;
            const MassRow m = mass_row<UNI>(a, node);
            if (m.any) {
                const int tn = t + 1 == a.N ? 0 : t + 1;
                const Stencil ln = load_stencil(a.L, node, sd, a.N, tn);
                R -= a.inv_tau * (mass_apply(m, l) - mass_apply(m, ln));
            }
            rr += R * R;
            gg += g * g;
        }
        rt[id] = (T)R;
    }
    block_pair_sum(rr, gg, a.part + 2 * (size_t)blockIdx.x);
}

// The linearised operator at the state U: (J v)^n = (M/tau)(v^n - v^{n-dir}) + K'(u^n) v^n with
// dir = +1 (J, eqs. (disc1)-(disc2) linearised) or -1 (J^T: the time coupling runs the other
// way, K' being symmetric). Writes out = J v when b is null and out = b - J v otherwise;
// boundary entries are 0. FP64 throughout. UNI as in k_adj_residual.
template <int LAW, bool UNI>
__global__ void __launch_bounds__(kBlock) k_jac_apply(AdjArgs a, const double* v, const double* b, double* out,
                                                      int dir) {
    const size_t total = a.nodes * (size_t)a.N;
    const size_t sd = a.side;
    for (size_t id = (size_t)virtual_block_of(blockIdx.x, gridDim.x, 1) * kBlock + threadIdx.x; id < total;
         id += (size_t)gridDim.x * kBlock) {
        size_t node = id >> a.lgN;
        if constexpr (UNI) node = (size_t)__builtin_amdgcn_readfirstlane((int)node);
        const int t = (int)(id & (size_t)(a.N - 1));
        const int i = (int)(node % sd), j = (int)(node / sd);
        double Jv = 0.0;
        const bool interior = i > 0 && j > 0 && i < a.n && j < a.n;
        if (interior) {
            const Stencil u = load_stencil(a.U, node, sd, a.N, t);
            const Stencil l = load_stencil(v, node, sd, a.N, t);
            const size_t c_ij = (size_t)j * a.n + i, c_w = c_ij - 1, c_s = c_ij - a.n, c_sw = c_ij - a.n - 1;
            const size_t tri[6] = {2 * c_ij, 2 * c_ij + 1, 2 * c_w, 2 * c_s + 1, 2 * c_sw, 2 * c_sw + 1};
            const double gux[6] = {u.e - u.c, u.ne - u.nn, u.c - u.w, u.e - u.c, u.s - u.sw, u.c - u.w};
            const double guy[6] = {u.ne - u.e, u.nn - u.c, u.nn - u.c, u.c - u.s, u.c - u.s, u.w - u.sw};
            const double glx[6] = {l.e - l.c, l.ne - l.nn, l.c - l.w, l.e - l.c, l.s - l.sw, l.c - l.w};
            const double gly[6] = {l.ne - l.e, l.nn - l.c, l.nn - l.c, l.c - l.s, l.c - l.s, l.w - l.sw};
            const int px[6] = {-1, 0, 1, -1, 0, 1};
            const int py[6] = {0, -1, -1, 1, 1, 0};
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                const double th = a.theta ? uload<UNI>(a.theta, tri[k]) : 1.0;
                const size_t rq = 4 * (size_t)region_of<UNI>(a, tri[k]);
                const double* rp = (const double*)a.regp;
                const double4 q = make_double4(uload<UNI>(rp, rq), uload<UNI>(rp, rq + 1), uload<UNI>(rp, rq + 2),
                                               uload<UNI>(rp, rq + 3));
                const Law L = tri_law_q<LAW>(q, a.n2, th, gux[k], guy[k]);
                Jv += tri_lin(L, gux[k], guy[k], glx[k], gly[k], px[k], py[k]);
            }
            const MassRow m = mass_row<UNI>(a, node);
            if (m.any) {
                const int to = dir > 0 ? (t == 0 ? a.N - 1 : t - 1) : (t + 1 == a.N ? 0 : t + 1);
                const Stencil lo = load_stencil(v, node, sd, a.N, to);
                Jv += a.inv_tau * (mass_apply(m, l) - mass_apply(m, lo));
            }
        }
        out[id] = interior ? (b ? b[id] - Jv : Jv) : 0.0;
    }
}

// One workgroup per cell (ci, cj), threads over time. Per triangle T of the cell:
//   gtheta_T = - sum_n |T| nuhat_T(|grad u^n|^2) grad u^n . grad lambda^n
//   gsigma_T = tau sum_n du^T M_T du - sum_n lambda^T M_T du,  du = (u^n - u^{n-1})/tau
//   loss_T   = sigma_T tau sum_n du^T M_T du
// with the unit-conductivity element mass |T|/12 (sum v w + sum v sum w), |T| = h^2 / 2.
// per_cell: write the sums over the two triangles of the cell instead of one value each.
template <int LAW>
__global__ void __launch_bounds__(kBlock) k_adj_grad(AdjArgs a, double* gth, double* gsg, int per_cell) {
    const int c = blockIdx.x;
    const int ci = c % a.n, cj = c / a.n;
    const size_t sd = a.side;
    const size_t v00 = (size_t)cj * sd + ci, v10 = v00 + 1, v11 = v00 + sd + 1, v01 = v00 + sd;
    const size_t NN = a.N;
    const int rg_a = a.flags[2 * c], rg_b = a.flags[2 * c + 1];
    const double h2_24 = 1.0 / (24.0 * a.n2);  // |T| / 12
    double th_acc[2] = {0.0, 0.0}, ss[2] = {0.0, 0.0}, ls[2] = {0.0, 0.0};
    for (int t = threadIdx.x; t < a.N; t += kBlock) {
        const int tp = t == 0 ? a.N - 1 : t - 1;
        const double u00 = a.U[v00 * NN + t], u10 = a.U[v10 * NN + t], u11 = a.U[v11 * NN + t],
                     u01 = a.U[v01 * NN + t];
        const double p00 = a.U[v00 * NN + tp], p10 = a.U[v10 * NN + tp], p11 = a.U[v11 * NN + tp],
                     p01 = a.U[v01 * NN + tp];
        const double d00 = (u00 - p00) * a.inv_tau, d10 = (u10 - p10) * a.inv_tau, d11 = (u11 - p11) * a.inv_tau,
                     d01 = (u01 - p01) * a.inv_tau;
        // T_a = {v00, v10, v11}, T_b = {v00, v11, v01}
        const double dsa = d00 + d10 + d11, dsb = d00 + d11 + d01;
        ss[0] += h2_24 * (d00 * d00 + d10 * d10 + d11 * d11 + dsa * dsa);
        ss[1] += h2_24 * (d00 * d00 + d11 * d11 + d01 * d01 + dsb * dsb);
        if (a.L) {
            const double l00 = a.L[v00 * NN + t], l10 = a.L[v10 * NN + t], l11 = a.L[v11 * NN + t],
                         l01 = a.L[v01 * NN + t];
            ls[0] += h2_24 * (l00 * d00 + l10 * d10 + l11 * d11 + (l00 + l10 + l11) * dsa);
            ls[1] += h2_24 * (l00 * d00 + l11 * d11 + l01 * d01 + (l00 + l11 + l01) * dsb);
            const double uax = u10 - u00, uay = u11 - u10, ubx = u11 - u01, uby = u01 - u00;
            const double lax = l10 - l00, lay = l11 - l10, lbx = l11 - l01, lby = l01 - l00;
            const Law La = tri_law<LAW>(a, rg_a, 1.0, uax, uay), Lb = tri_law<LAW>(a, rg_b, 1.0, ubx, uby);
            th_acc[0] += 0.5 * La.nu * (uax * lax + uay * lay);
            th_acc[1] += 0.5 * Lb.nu * (ubx * lbx + uby * lby);
        }
    }
    // fixed-order workgroup sums of the six accumulators
    __shared__ double red[6][kBlock];
    red[0][threadIdx.x] = th_acc[0];
    red[1][threadIdx.x] = th_acc[1];
    red[2][threadIdx.x] = ss[0];
    red[3][threadIdx.x] = ss[1];
    red[4][threadIdx.x] = ls[0];
    red[5][threadIdx.x] = ls[1];
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int q = 0; q < 6; ++q) red[q][threadIdx.x] += red[q][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double gta = -red[0][0], gtb = -red[1][0];
        const double gsa = a.tau * red[2][0] - red[4][0], gsb = a.tau * red[3][0] - red[5][0];
        const double loss = a.tau * (a.sig[2 * c] * red[2][0] + a.sig[2 * c + 1] * red[3][0]);
        if (per_cell) {
            if (gth) gth[c] = gta + gtb;
            if (gsg) gsg[c] = gsa + gsb;
        } else {
            if (gth) {
                gth[2 * c] = gta;
                gth[2 * c + 1] = gtb;
            }
            if (gsg) {
                gsg[2 * c] = gsa;
                gsg[2 * c + 1] = gsb;
            }
        }
        a.part[2 * (size_t)c] = loss;
        a.part[2 * (size_t)c + 1] = 0.0;
    }
}

static AdjArgs mk_adj(const Plan& p, char* ws) {
    AdjArgs a;
    a.n = p.n;
    a.side = p.side;
    a.N = p.N;
    a.lgN = 0;
    while ((1 << a.lgN) < p.N) ++a.lgN;
    a.nodes = p.nodes;
    a.tau = p.tau;
    a.inv_tau = 1.0 / p.tau;
    a.n2 = (double)p.n * (double)p.n;
    a.regp = (const double4*)(ws + p.off_regp);
    a.U = (const double*)(ws + p.off_U);
    a.L = (const double*)(ws + p.off_L);
    a.G = (const double*)(ws + p.off_G);
    a.mt = (const double*)(ws + p.lev[0].off_mt);
    a.flags = (const uint8_t*)(ws + p.off_flags);
    a.theta = p.prob.d_theta;
    a.sig = (const double*)(ws + p.off_sig);
    a.part = (double*)(ws + p.off_part);
    return a;
}

// Grid of the grid-stride kernels over [nodes][N]: a multiple of kNumXcd workgroups, remapped
// (virtual_block_of) so that every XCD walks contiguous node ranges and finds the stencil
// neighbours of its nodes in its own L2.
static_assert(kAdjBlocks % kNumXcd == 0, "the adjoint grid is a multiple of the XCD count");
static int adj_grid(size_t total) {
    size_t g = (total + kBlock - 1) / kBlock;
    g = (g + kNumXcd - 1) / kNumXcd * kNumXcd;
    if (g > (size_t)kAdjBlocks) g = kAdjBlocks;
    return (int)g;
}

void launch_adj_source(const Plan& p, char* ws, hipStream_t st) {
    AdjArgs a = mk_adj(p, ws);
    hipLaunchKernelGGL(k_adj_source, dim3(adj_grid(p.nodes * p.N)), dim3(kBlock), 0, st, a, (double*)(ws + p.off_G));
}

template <typename X> struct AdjTag {
    using type = X;
};

int launch_adj_residual(const Plan& p, char* ws, void* rt, hipStream_t st) {
    AdjArgs a = mk_adj(p, ws);
    const int grid = adj_grid(p.nodes * p.N);
    const bool ex = p.law == PT_NU_EXPCAP;
    auto go = [&](auto t_, auto uni_) {
        using T = typename decltype(t_)::type;
        constexpr bool U = decltype(uni_)::value;
        if (ex)
            hipLaunchKernelGGL((k_adj_residual<T, PT_NU_EXPCAP, U>), dim3(grid), dim3(kBlock), 0, st, a, (T*)rt);
        else
            hipLaunchKernelGGL((k_adj_residual<T, PT_NU_RATIONAL, U>), dim3(grid), dim3(kBlock), 0, st, a, (T*)rt);
    };
    const bool uni = p.N >= 64;   // one node per wavefront
    if (p.fp32) {
        if (uni) go(AdjTag<float>(), std::true_type());
        else go(AdjTag<float>(), std::false_type());
    } else {
        if (uni) go(AdjTag<double>(), std::true_type());
        else go(AdjTag<double>(), std::false_type());
    }
    return grid;
}

void launch_adj_grad(const Plan& p, char* ws, bool with_lambda, double* gth, double* gsg, int per_cell,
                     hipStream_t st) {
    AdjArgs a = mk_adj(p, ws);
    if (!with_lambda) a.L = nullptr;
    const dim3 grid((unsigned)p.n * (unsigned)p.n);
    if (p.law == PT_NU_EXPCAP)
        hipLaunchKernelGGL(k_adj_grad<PT_NU_EXPCAP>, grid, dim3(kBlock), 0, st, a, gth, gsg, per_cell);
    else
        hipLaunchKernelGGL(k_adj_grad<PT_NU_RATIONAL>, grid, dim3(kBlock), 0, st, a, gth, gsg, per_cell);
}

void launch_jac_apply(const Plan& p, char* ws, const double* v, const double* b, double* out, int dir,
                      hipStream_t st) {
    AdjArgs a = mk_adj(p, ws);
    const dim3 grid(adj_grid(p.nodes * p.N));
    const bool ex = p.law == PT_NU_EXPCAP, uni = p.N >= 64;
    if (ex && uni)
        hipLaunchKernelGGL((k_jac_apply<PT_NU_EXPCAP, true>), grid, dim3(kBlock), 0, st, a, v, b, out, dir);
    else if (ex)
        hipLaunchKernelGGL((k_jac_apply<PT_NU_EXPCAP, false>), grid, dim3(kBlock), 0, st, a, v, b, out, dir);
    else if (uni)
        hipLaunchKernelGGL((k_jac_apply<PT_NU_RATIONAL, true>), grid, dim3(kBlock), 0, st, a, v, b, out, dir);
    else
        hipLaunchKernelGGL((k_jac_apply<PT_NU_RATIONAL, false>), grid, dim3(kBlock), 0, st, a, v, b, out, dir);
}

}  // namespace pt
