// Frequency-domain kernels: the batched solve of the complex-shifted systems
//     A_s x_s = (Khat + z_s M) x_s = r_s,   z_s = (1 - exp(-2 pi i s / N)) / tau,
// one per frequency slot (remark rem:parallel: the DFT in time block-diagonalises the
// periodic, time-invariant linear problem of eqs. (iter1)-(iter2)). All slots of all
// nodes are processed in one launch; thread (node, slot), slots fastest.
//
// Operators on a level with side points per row (interior nodes only; vectors are zero
// on the boundary):
//   Khat x = nu_max (4 x_c - x_e - x_w - x_n - x_s)       (P1 stiffness on this grid)
//   M x    = 7-point stencil from the level's table (c, e, n, ne, and symmetry)
// Multigrid: damped Jacobi smoothing with D = 4 nu_max + z diag(M), P1 interpolation P
// between nested grids, restriction P^T, Galerkin coarse mass (k_setup.hip), exact solve
// on the 2 x 2-cell grid (one unknown). One V(1,1) cycle is symmetric (B^T = B).
#include "pt_device.h"

namespace pt {

struct LvArgs {
    int n, side;
    size_t nodes;
    const double* mt;
};

struct SlotArgs {
    int S, steps, per_step, slot_chunk, remap;
    double nu, omega;
    const double* zs;  // S x 3 generic (a, b, c) of the shifts
};

__device__ __forceinline__ LvArgs mk_lv(const LevelDesc& d, char* ws) {
    LvArgs l;
    l.n = d.n;
    l.side = d.side;
    l.nodes = d.nodes;
    l.mt = (const double*)(ws + d.off_mt);
    return l;
}

template <typename T> __device__ __forceinline__ GS<T> load_shift(const double* zs, int s) {
    GS<T> g;
    g.a = (T)zs[3 * s];
    g.b = (T)zs[3 * s + 1];
    g.c = (T)zs[3 * s + 2];
    return g;
}

// (A x)_a for interior node a, given the 7 neighbour values of x.
template <typename T, typename T2>
__device__ __forceinline__ T2 apply_A(const LvArgs& L, size_t a, T nu, const GS<T>& z, T2 xc, T2 xe, T2 xw, T2 xn,
                                      T2 xs, T2 xne, T2 xsw) {
    const size_t nd = L.nodes, sd = L.side;
    T2 Lx;
    Lx.x = nu * ((T)4 * xc.x - xe.x - xw.x - xn.x - xs.x);
    Lx.y = nu * ((T)4 * xc.y - xe.y - xw.y - xn.y - xs.y);
    T mc = (T)L.mt[a], me = (T)L.mt[nd + a], mw = (T)L.mt[nd + a - 1], mn = (T)L.mt[2 * nd + a],
      ms = (T)L.mt[2 * nd + a - sd], mne = (T)L.mt[3 * nd + a], msw = (T)L.mt[3 * nd + a - sd - 1];
    T2 Mx = scale2(mc, xc);
    Mx = fma2(me, xe, Mx);
    Mx = fma2(mw, xw, Mx);
    Mx = fma2(mn, xn, Mx);
    Mx = fma2(ms, xs, Mx);
    Mx = fma2(mne, xne, Mx);
    Mx = fma2(msw, xsw, Mx);
    return add2(Lx, gs_apply(z, Mx));
}

// ---------------------------------------------------------------- dot-product partials

// Reduce the per-thread partial sums of a workgroup over threads sharing a slot and
// store them at part[(vb * S + s) * 3 + c].
__device__ __forceinline__ void store_dot_partials(const double* acc, double* part, int vb, int S, int chunk, int SC) {
    __shared__ double red[3][kBlock];
    red[0][threadIdx.x] = acc[0];
    red[1][threadIdx.x] = acc[1];
    red[2][threadIdx.x] = acc[2];
    __syncthreads();
    if ((int)threadIdx.x < SC) {
        double s0 = 0, s1 = 0, s2 = 0;
        for (int t = threadIdx.x; t < kBlock; t += SC) {
            s0 += red[0][t];
            s1 += red[1][t];
            s2 += red[2][t];
        }
        size_t s = (size_t)chunk * SC + threadIdx.x;
        double* o = part + ((size_t)vb * S + s) * 3;
        o[0] = s0;
        o[1] = s1;
        o[2] = s2;
    }
}

// ---------------------------------------------------------------- V-cycle: down

// r_c = P^T (r - A x1) with the pre-smoothed x1 = omega D^{-1} r (one Jacobi sweep from
// zero), evaluated per coarse node from the fine values on the 2-ring around its fine
// twin (19 nodes).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_vc_down(SlotArgs sa, LvArgs F, LvArgs C, const void* rin_, void* rout_) {
    using T2 = typename Vec2<T>::type;
    const T2* rin = (const T2*)rin_;
    T2* rout = (T2*)rout_;
    const int S = sa.S, SC = sa.slot_chunk;
    const int ls = threadIdx.x % SC, ln = threadIdx.x / SC;
    const int s = blockIdx.y * SC + ls;
    const int vb = virtual_block(sa.remap);
    const GS<T> z = load_shift<T>(sa.zs, s);
    const T nu = (T)sa.nu, om = (T)sa.omega, dl = (T)4 * nu;
    const long sf = F.side;
    for (int step = 0; step < sa.steps; ++step) {
        size_t I = ((size_t)vb * sa.steps + step) * sa.per_step + ln;
        if (I >= C.nodes) continue;
        int ci = (int)(I % C.side), cj = (int)(I / C.side);
        T2 out = mk2<T>(0, 0);
        if (ci > 0 && cj > 0 && ci < C.n && cj < C.n) {
            size_t c = (size_t)(2 * cj) * sf + 2 * ci;
            // x1 on the 5 x 5 patch around c (only the 19 hexagonal-ring points are used)
            T2 x1[5][5];
#pragma unroll
            for (int dy = -2; dy <= 2; ++dy) {
#pragma unroll
                for (int dx = -2; dx <= 2; ++dx) {
                    int ddx = dx - dy;
                    bool need = (ddx >= -2 && ddx <= 2) && !((dx == 2 && dy == -2) || (dx == -2 && dy == 2));
                    // hexagonal distance in the SW-NE lattice: max(|dx|,|dy|,|dx-dy|) <= 2
                    need = need && (dx >= -2 && dx <= 2 && dy >= -2 && dy <= 2);
                    if (need) {
                        size_t b = c + (long)dy * sf + dx;
                        T2 rb = rin[b * S + s];
                        GS<T> di = gs_inv_diag<T>(dl, (T)F.mt[b], z);
                        x1[dy + 2][dx + 2] = scale2(om, gs_apply(di, rb));
                    } else {
                        x1[dy + 2][dx + 2] = mk2<T>(0, 0);
                    }
                }
            }
            // supports of the coarse hat function: offset and weight
            const int ox[7] = {0, 1, -1, 0, 0, 1, -1};
            const int oy[7] = {0, 0, 0, 1, -1, 1, -1};
#pragma unroll
            for (int q = 0; q < 7; ++q) {
                int X = ox[q] + 2, Y = oy[q] + 2;
                size_t a = c + (long)oy[q] * sf + ox[q];
                T2 Ax = apply_A<T, T2>(F, a, nu, z, x1[Y][X], x1[Y][X + 1], x1[Y][X - 1], x1[Y + 1][X], x1[Y - 1][X],
                                       x1[Y + 1][X + 1], x1[Y - 1][X - 1]);
                T2 res = sub2(rin[a * S + s], Ax);
                out = fma2(q == 0 ? (T)1 : (T)0.5, res, out);
            }
        }
        rout[I * S + s] = out;
    }
}

// ---------------------------------------------------------------- V-cycle: coarsest

// Exact solve on the 2 x 2-cell grid: the single interior node (1, 1) has the 1 x 1
// operator 4 nu_max + z M_c.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_vc_coarsest(SlotArgs sa, LvArgs C, const void* rin_, void* xout_) {
    using T2 = typename Vec2<T>::type;
    const T2* rin = (const T2*)rin_;
    T2* xout = (T2*)xout_;
    const int S = sa.S;
    for (int s = blockIdx.x * kBlock + threadIdx.x; s < S; s += gridDim.x * kBlock) {
        const GS<T> z = load_shift<T>(sa.zs, s);
        for (size_t node = 0; node < C.nodes; ++node) {
            T2 v = mk2<T>(0, 0);
            if (node == (size_t)C.side + 1) {
                GS<T> di = gs_inv_diag<T>((T)4 * (T)sa.nu, (T)C.mt[node], z);
                v = gs_apply(di, rin[node * S + s]);
            }
            xout[node * S + s] = v;
        }
    }
}

// ---------------------------------------------------------------- V-cycle: up

template <typename T2>
__device__ __forceinline__ T2 prolong_at(const T2* xc, int sc, int S, int s, int bi, int bj) {
    int hi = bi >> 1, hj = bj >> 1;
    bool oi = bi & 1, oj = bj & 1;
    if (!oi && !oj) return xc[((size_t)hj * sc + hi) * S + s];
    T2 p, q;
    if (oi && !oj) {
        p = xc[((size_t)hj * sc + hi) * S + s];
        q = xc[((size_t)hj * sc + hi + 1) * S + s];
    } else if (!oi && oj) {
        p = xc[((size_t)hj * sc + hi) * S + s];
        q = xc[((size_t)(hj + 1) * sc + hi) * S + s];
    } else {
        p = xc[((size_t)hj * sc + hi) * S + s];
        q = xc[((size_t)(hj + 1) * sc + hi + 1) * S + s];
    }
    T2 r;
    r.x = (p.x + q.x) * 0.5f;
    r.y = (p.y + q.y) * 0.5f;
    return r;
}

// x2 = omega D^{-1} r + P x_c (pre-smoothed iterate plus coarse correction), then one
// post-smoothing sweep x3 = x2 + omega D^{-1} (r - A x2). Optionally accumulates the
// dot partials of (x3, r).
template <typename T>
__global__ void __launch_bounds__(kBlock) k_vc_up(SlotArgs sa, LvArgs F, LvArgs C, const void* rin_,
                                                  const void* xc_, void* xout_, int dotmode, double* part) {
    using T2 = typename Vec2<T>::type;
    const T2* rin = (const T2*)rin_;
    const T2* xc = (const T2*)xc_;
    T2* xout = (T2*)xout_;
    const int S = sa.S, SC = sa.slot_chunk;
    const int ls = threadIdx.x % SC, ln = threadIdx.x / SC;
    const int s = blockIdx.y * SC + ls;
    const int vb = virtual_block(sa.remap);
    const GS<T> z = load_shift<T>(sa.zs, s);
    const T nu = (T)sa.nu, om = (T)sa.omega, dl = (T)4 * nu;
    const long sf = F.side;
    double acc[3] = {0, 0, 0};
    for (int step = 0; step < sa.steps; ++step) {
        size_t a = ((size_t)vb * sa.steps + step) * sa.per_step + ln;
        if (a >= F.nodes) continue;
        int ai = (int)(a % F.side), aj = (int)(a / F.side);
        T2 out = mk2<T>(0, 0);
        if (ai > 0 && aj > 0 && ai < F.n && aj < F.n) {
            const int ox[7] = {0, 1, -1, 0, 0, 1, -1};
            const int oy[7] = {0, 0, 0, 1, -1, 1, -1};
            T2 x2[7];
            T2 ra;
#pragma unroll
            for (int q = 0; q < 7; ++q) {
                size_t b = a + (long)oy[q] * sf + ox[q];
                T2 rb = rin[b * S + s];
                if (q == 0) ra = rb;
                GS<T> di = gs_inv_diag<T>(dl, (T)F.mt[b], z);
                T2 v = scale2(om, gs_apply(di, rb));
                x2[q] = add2(v, prolong_at(xc, C.side, S, s, ai + ox[q], aj + oy[q]));
            }
            T2 Ax = apply_A<T, T2>(F, a, nu, z, x2[0], x2[1], x2[2], x2[3], x2[4], x2[5], x2[6]);
            GS<T> da = gs_inv_diag<T>(dl, (T)F.mt[a], z);
            out = add2(x2[0], scale2(om, gs_apply(da, sub2(ra, Ax))));
            if (dotmode != DOT_NONE) dot3_acc(acc, out, ra, dotmode == DOT_HERM);
        }
        xout[a * S + s] = out;
    }
    if (dotmode != DOT_NONE) store_dot_partials(acc, part, vb, S, blockIdx.y, SC);
}

// ---------------------------------------------------------------- operator apply

template <typename T>
__global__ void __launch_bounds__(kBlock) k_matvec(SlotArgs sa, LvArgs F, const void* x_, void* y_, int dotmode,
                                                   double* part) {
    using T2 = typename Vec2<T>::type;
    const T2* x = (const T2*)x_;
    T2* y = (T2*)y_;
    const int S = sa.S, SC = sa.slot_chunk;
    const int ls = threadIdx.x % SC, ln = threadIdx.x / SC;
    const int s = blockIdx.y * SC + ls;
    const int vb = virtual_block(sa.remap);
    const GS<T> z = load_shift<T>(sa.zs, s);
    const T nu = (T)sa.nu;
    const long sf = F.side;
    double acc[3] = {0, 0, 0};
    for (int step = 0; step < sa.steps; ++step) {
        size_t a = ((size_t)vb * sa.steps + step) * sa.per_step + ln;
        if (a >= F.nodes) continue;
        int ai = (int)(a % F.side), aj = (int)(a / F.side);
        T2 out = mk2<T>(0, 0);
        if (ai > 0 && aj > 0 && ai < F.n && aj < F.n) {
            T2 xc = x[a * S + s];
            out = apply_A<T, T2>(F, a, nu, z, xc, x[(a + 1) * S + s], x[(a - 1) * S + s], x[(a + sf) * S + s],
                                 x[(a - sf) * S + s], x[(a + sf + 1) * S + s], x[(a - sf - 1) * S + s]);
            if (dotmode != DOT_NONE) dot3_acc(acc, xc, out, dotmode == DOT_HERM);
        }
        if (y) y[a * S + s] = out;
    }
    if (dotmode != DOT_NONE) store_dot_partials(acc, part, vb, S, blockIdx.y, SC);
}

// ---------------------------------------------------------------- per-slot scalars

// Sum the partials of every workgroup in a fixed order and combine them into a generic
// scalar: Hermitian u^H v = (s1 + s2) + i s3, bilinear u^T v = (s1 - s2) + i s3, and for
// slot 0 the two real dot products (s1, s2).
__global__ void __launch_bounds__(kBlock) k_reduce_dots(const double* part, int nblk, int S, int herm, double* out) {
    for (int s = blockIdx.x * kBlock + threadIdx.x; s < S; s += gridDim.x * kBlock) {
        double s1 = 0, s2 = 0, s3 = 0;
        for (int b = 0; b < nblk; ++b) {
            const double* o = part + ((size_t)b * S + s) * 3;
            s1 += o[0];
            s2 += o[1];
            s3 += o[2];
        }
        double2 r;
        if (s == 0) {
            r.x = s1;
            r.y = s2;
        } else {
            r.x = herm ? (s1 + s2) : (s1 - s2);
            r.y = s3;
        }
        ((double2*)out)[s] = r;
    }
}

// coef = num / den in generic arithmetic. A zero denominator with a zero numerator (a
// frequency whose right-hand side vanishes) gives 0; a vanishing denominator with a
// nonzero numerator sets *flag (COCG breakdown) and gives 0.
__global__ void __launch_bounds__(kBlock) k_slot_div(const double* num_, const double* den_, double* coef_, int S,
                                                     int* flag) {
    const double2* num = (const double2*)num_;
    const double2* den = (const double2*)den_;
    double2* coef = (double2*)coef_;
    for (int s = blockIdx.x * kBlock + threadIdx.x; s < S; s += gridDim.x * kBlock) {
        double2 a = num[s], b = den[s], r;
        if (s == 0) {
            r.x = (b.x != 0.0) ? a.x / b.x : 0.0;
            r.y = (b.y != 0.0) ? a.y / b.y : 0.0;
            if (flag && ((b.x == 0.0 && a.x != 0.0) || (b.y == 0.0 && a.y != 0.0))) *flag = 1;
        } else {
            double d = b.x * b.x + b.y * b.y;
            if (d != 0.0) {
                r.x = (a.x * b.x + a.y * b.y) / d;
                r.y = (a.y * b.x - a.x * b.y) / d;
            } else {
                r.x = 0.0;
                r.y = 0.0;
                if (flag && (a.x != 0.0 || a.y != 0.0)) *flag = 1;
            }
        }
        coef[s] = r;
    }
}

// ---------------------------------------------------------------- COCG vector updates

template <typename T>
__global__ void __launch_bounds__(kBlock) k_cocg_xr(int S, size_t total, const double* coef, void* x_, void* r_,
                                                    const void* p_, const void* q_) {
    using T2 = typename Vec2<T>::type;
    T2* x = (T2*)x_;
    T2* r = (T2*)r_;
    const T2* p = (const T2*)p_;
    const T2* q = (const T2*)q_;
    for (size_t id = blockIdx.x * (size_t)kBlock + threadIdx.x; id < total; id += (size_t)gridDim.x * kBlock) {
        int s = (int)(id % S);
        GS<T> g = gs_from<T>(((const double2*)coef)[s], s == 0);
        x[id] = add2(x[id], gs_apply(g, p[id]));
        r[id] = sub2(r[id], gs_apply(g, q[id]));
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_cocg_p(int S, size_t total, const double* coef, const void* z_, void* p_) {
    using T2 = typename Vec2<T>::type;
    const T2* z = (const T2*)z_;
    T2* p = (T2*)p_;
    for (size_t id = blockIdx.x * (size_t)kBlock + threadIdx.x; id < total; id += (size_t)gridDim.x * kBlock) {
        int s = (int)(id % S);
        GS<T> g = gs_from<T>(((const double2*)coef)[s], s == 0);
        p[id] = add2(z[id], gs_apply(g, p[id]));
    }
}

// ---------------------------------------------------------------- host launchers

static SlotArgs mk_slot(const Plan& p, char* ws, const Geom& g) {
    SlotArgs sa;
    sa.S = p.S;
    sa.steps = g.steps;
    sa.per_step = g.per_step;
    sa.slot_chunk = g.slot_chunk;
    sa.remap = p.opt.xcd_remap;
    sa.nu = p.prob.nu_max;
    sa.omega = p.opt.vc_omega;
    sa.zs = (const double*)(ws + p.off_zs);
    return sa;
}

static LvArgs host_lv(const Plan& p, char* ws, int l) {
    LvArgs L;
    L.n = p.lev[l].n;
    L.side = p.lev[l].side;
    L.nodes = p.lev[l].nodes;
    L.mt = (const double*)(ws + p.lev[l].off_mt);
    return L;
}

static int flat_grid(size_t total) {
    size_t g = (total + kBlock - 1) / kBlock;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (int)g;
}

void launch_vcycle(const Plan& p, char* ws, const void* r0, void* x0, int dotmode, double* part, hipStream_t st) {
    const int L = p.nlev;
    // restriction sweep
    for (int l = 0; l + 1 < L; ++l) {
        const void* rin = (l == 0) ? r0 : (const void*)(ws + p.lev[l].off_r);
        void* rout = ws + p.lev[l + 1].off_r;
        Geom g = slot_geom(p.lev[l + 1].nodes, p.S);
        SlotArgs sa = mk_slot(p, ws, g);
        dim3 grid(g.blocks, g.chunks);
        int kid = (l == 0) ? KID_DOWN0 : KID_DOWNC;
        tm_begin(p, kid, st);
        if (p.fp32)
            hipLaunchKernelGGL(k_vc_down<float>, grid, dim3(kBlock), 0, st, sa, host_lv(p, ws, l), host_lv(p, ws, l + 1),
                               rin, rout);
        else
            hipLaunchKernelGGL(k_vc_down<double>, grid, dim3(kBlock), 0, st, sa, host_lv(p, ws, l),
                               host_lv(p, ws, l + 1), rin, rout);
        tm_end(p, kid, st);
    }
    {
        Geom g = slot_geom(p.lev[L - 1].nodes, p.S);
        SlotArgs sa = mk_slot(p, ws, g);
        const void* rin = (L == 1) ? r0 : (const void*)(ws + p.lev[L - 1].off_r);
        void* xout = (L == 1) ? x0 : (void*)(ws + p.lev[L - 1].off_x);
        int grid = (p.S + kBlock - 1) / kBlock;
        tm_begin(p, KID_COARSEST, st);
        if (p.fp32)
            hipLaunchKernelGGL(k_vc_coarsest<float>, dim3(grid), dim3(kBlock), 0, st, sa, host_lv(p, ws, L - 1), rin, xout);
        else
            hipLaunchKernelGGL(k_vc_coarsest<double>, dim3(grid), dim3(kBlock), 0, st, sa, host_lv(p, ws, L - 1), rin,
                               xout);
        tm_end(p, KID_COARSEST, st);
    }
    // prolongation sweep
    for (int l = L - 2; l >= 0; --l) {
        const void* rin = (l == 0) ? r0 : (const void*)(ws + p.lev[l].off_r);
        void* xout = (l == 0) ? x0 : (void*)(ws + p.lev[l].off_x);
        const void* xc = ws + p.lev[l + 1].off_x;
        Geom g = slot_geom(p.lev[l].nodes, p.S);
        SlotArgs sa = mk_slot(p, ws, g);
        dim3 grid(g.blocks, g.chunks);
        int dm = (l == 0) ? dotmode : DOT_NONE;
        int kid = (l == 0) ? KID_UP0 : KID_UPC;
        tm_begin(p, kid, st);
        if (p.fp32)
            hipLaunchKernelGGL(k_vc_up<float>, grid, dim3(kBlock), 0, st, sa, host_lv(p, ws, l), host_lv(p, ws, l + 1),
                               rin, xc, xout, dm, part);
        else
            hipLaunchKernelGGL(k_vc_up<double>, grid, dim3(kBlock), 0, st, sa, host_lv(p, ws, l), host_lv(p, ws, l + 1),
                               rin, xc, xout, dm, part);
        tm_end(p, kid, st);
    }
}

void launch_matvec(const Plan& p, char* ws, const void* x, void* y, int dotmode, double* part, hipStream_t st) {
    const Geom& g = p.g_slot0;
    SlotArgs sa = mk_slot(p, ws, g);
    dim3 grid(g.blocks, g.chunks);
    if (p.fp32)
        hipLaunchKernelGGL(k_matvec<float>, grid, dim3(kBlock), 0, st, sa, host_lv(p, ws, 0), x, y, dotmode, part);
    else
        hipLaunchKernelGGL(k_matvec<double>, grid, dim3(kBlock), 0, st, sa, host_lv(p, ws, 0), x, y, dotmode, part);
}

void launch_reduce_dots(const Plan& p, double* part, int dotmode, double* out, hipStream_t st) {
    int grid = (p.S + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_reduce_dots, dim3(grid), dim3(kBlock), 0, st, (const double*)part, p.g_slot0.blocks, p.S,
                       dotmode == DOT_HERM ? 1 : 0, out);
}

void launch_slot_div(const Plan& p, const double* num, const double* den, double* coef, int* flag, hipStream_t st) {
    int grid = (p.S + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_slot_div, dim3(grid), dim3(kBlock), 0, st, num, den, coef, p.S, flag);
}

void launch_cocg_xr(const Plan& p, const double* coef, void* x, void* r, const void* pv, const void* q,
                    hipStream_t st) {
    size_t total = p.nodes * (size_t)p.S;
    if (p.fp32)
        hipLaunchKernelGGL(k_cocg_xr<float>, dim3(flat_grid(total)), dim3(kBlock), 0, st, p.S, total, coef, x, r, pv, q);
    else
        hipLaunchKernelGGL(k_cocg_xr<double>, dim3(flat_grid(total)), dim3(kBlock), 0, st, p.S, total, coef, x, r, pv,
                           q);
}

void launch_cocg_p(const Plan& p, const double* coef, const void* z, void* pv, hipStream_t st) {
    size_t total = p.nodes * (size_t)p.S;
    if (p.fp32)
        hipLaunchKernelGGL(k_cocg_p<float>, dim3(flat_grid(total)), dim3(kBlock), 0, st, p.S, total, coef, z, pv);
    else
        hipLaunchKernelGGL(k_cocg_p<double>, dim3(flat_grid(total)), dim3(kBlock), 0, st, p.S, total, coef, z, pv);
}

void launch_copy_slots(const Plan& p, const void* src, void* dst, hipStream_t st) {
    hipMemcpyAsync(dst, src, p.nodes * (size_t)p.S * p.elem, hipMemcpyDeviceToDevice, st);
}

}  // namespace pt
