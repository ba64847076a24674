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

// S: slots per instance (a power of two; slot s with s % S == 0 packs k = 0 and k = N/2),
// ST = B S: slots per node over the B instances of a batch (the row stride).
struct SlotArgs {
    int S, ST, lgST, per_step, slot_chunk, remap, col_groups, rows_per_chunk;
    double nu, omega;
    const double* zs;  // S x 3 generic (a, b, c) of the shifts
};

template <typename T> __device__ __forceinline__ GS<T> load_shift(const double* zs, int s) {
    GS<T> g;
    g.a = (T)zs[3 * s];
    g.b = (T)zs[3 * s + 1];
    g.c = (T)zs[3 * s + 2];
    return g;
}

// Addressing: a workgroup walks the same grid row in all its threads, so row base
// pointers are uniform; per-lane positions inside a row are loop-invariant 32-bit byte
// offsets (a row holds at most 4097 x 512 slot values).
template <typename P> __device__ __forceinline__ const P* cboff(const P* base, unsigned bytes) {
    return reinterpret_cast<const P*>(reinterpret_cast<const char*>(base) + bytes);
}
template <typename P> __device__ __forceinline__ P* boff(P* base, unsigned bytes) {
    return reinterpret_cast<P*>(reinterpret_cast<char*>(base) + bytes);
}
// Row `row` of a slot vector with `side` nodes per row and 2^lgST slots per node.
template <typename P> __device__ __forceinline__ P* row_of(P* base, int row, int side, int lgST) {
    return base + ((size_t)(row * side) << lgST);
}

// The seven mass-stencil coefficients of node a (centre, E, W, N, S, NE, SW).
struct MRow {
    double c, e, w, n, s, ne, sw;
    __device__ __forceinline__ bool any() const {
        return c != 0.0 || e != 0.0 || w != 0.0 || n != 0.0 || s != 0.0 || ne != 0.0 || sw != 0.0;
    }
};

__device__ __forceinline__ MRow mrow(const LvArgs& L, long a) {
    const long nd = (long)L.nodes, sd = L.side;
    MRow m;
    m.c = L.mt[a];
    m.e = L.mt[nd + a];
    m.w = L.mt[nd + a - 1];
    m.n = L.mt[2 * nd + a];
    m.s = L.mt[2 * nd + a - sd];
    m.ne = L.mt[3 * nd + a];
    m.sw = L.mt[3 * nd + a - sd - 1];
    return m;
}

// (A x)_a for interior node a with mass row m, given the 7 neighbour values of x.
template <typename T, typename T2>
__device__ __forceinline__ T2 apply_A(const MRow& m, T nu, const GS<T>& z, T2 xc, T2 xe, T2 xw, T2 xn, T2 xs,
                                      T2 xne, T2 xsw) {
    T2 Lx;
    Lx.x = nu * ((T)4 * xc.x - xe.x - xw.x - xn.x - xs.x);
    Lx.y = nu * ((T)4 * xc.y - xe.y - xw.y - xn.y - xs.y);
    if (!m.any()) return Lx;
    T2 Mx = scale2((T)m.c, xc);
    Mx = fma2((T)m.e, xe, Mx);
    Mx = fma2((T)m.w, xw, Mx);
    Mx = fma2((T)m.n, xn, Mx);
    Mx = fma2((T)m.s, xs, Mx);
    Mx = fma2((T)m.ne, xne, Mx);
    Mx = fma2((T)m.sw, xsw, Mx);
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
// zero). Thread (coarse column ci, slot) walks up the fine rows R around fine column
// c = 2 ci with a 3-row x 5-column register window of x1 (rows R-1..R+1, columns
// c-2..c+2), forms the fine residual s = r - A x1 at columns c-1, c, c+1 of row R and adds
// it into the coarse rows it belongs to with the P^T weights: row 2cj-1 contributes
// (c-1, c) x 1/2, row 2cj contributes (c-1, c, c+1) x (1/2, 1, 1/2), row 2cj+1
// contributes (c, c+1) x 1/2 (P1 interpolation on the SW-NE split grid). The inputs of
// row R+2 are loaded before row R is computed.
template <typename T, bool UNI>
__global__ void __launch_bounds__(kBlock) k_vc_down(SlotArgs sa, LvArgs F, LvArgs C, const void* rin_, void* rout_) {
    using T2 = typename Vec2<T>::type;
    const T2* rin = (const T2*)rin_;
    T2* rout = (T2*)rout_;
    const int ST = sa.ST, lgST = sa.lgST, SC = sa.slot_chunk;
    const int ls = threadIdx.x % SC, ln = threadIdx.x / SC;
    const int s = blockIdx.y * SC + ls;
    const int vb = virtual_block(sa.remap);
    const GS<T> z = load_shift<T>(sa.zs, s);
    const T nu = (T)sa.nu, om = (T)sa.omega, dl = (T)4 * nu, idl = (T)1 / dl;
    const int sf = F.side, nF = F.n, sc = C.side, nc = C.n;
    const long nd = (long)F.nodes;
    const T half = (T)0.5;
    const unsigned E = sizeof(T2);
    const SweepRange sr = sweep_range(vb, sa.col_groups, sa.per_step, sa.rows_per_chunk, sc);
    int ci = sr.col0 + ln;
    if (UNI) ci = __builtin_amdgcn_readfirstlane(ci);
    if (ci >= sc) return;
    const T2 zero = mk2<T>(0, 0);
    const unsigned oco = (((unsigned)ci << lgST) + s) * E;
    // boundary coarse nodes of this chunk are zero
    for (int cj = sr.row0; cj < sr.row1; ++cj)
        if (ci == 0 || ci == nc || cj == 0 || cj == nc) *boff(row_of(rout, cj, sc, lgST), oco) = zero;
    if (ci == 0 || ci == nc) return;
    const int cj0 = sr.row0 > 1 ? sr.row0 : 1;
    const int cj1 = sr.row1 < nc ? sr.row1 : nc;  // interior coarse rows [cj0, cj1)
    if (cj0 >= cj1) return;
    const int c = 2 * ci;
    unsigned of[5];
#pragma unroll
    for (int d = 0; d < 5; ++d) of[d] = (((unsigned)(c - 2 + d) << lgST) + s) * E;
    // x1 and r on fine row R, columns c-2..c+2 (r kept for the three centre columns)
    T2 xa[5], xb[5], xq[5], rb[3], rq[3];
    auto fetch_row = [&](int R, T2* rv, double* mv) {
        if (R >= 0 && R <= nF) {
            const T2* fr = row_of(rin, R, sf, lgST);
            const double* mr = F.mt + (long)R * sf + (c - 2);
#pragma unroll
            for (int d = 0; d < 5; ++d) {
                rv[d] = *cboff(fr, of[d]);
                mv[d] = mr[d];
            }
        } else {
#pragma unroll
            for (int d = 0; d < 5; ++d) {
                rv[d] = zero;
                mv[d] = 0.0;
            }
        }
    };
    auto eval_row = [&](const T2* rv, const double* mv, T2* xr, T2* rr) {
#pragma unroll
        for (int d = 0; d < 5; ++d) {
            GS<T> di = gs_inv_diag<T>(dl, idl, (T)mv[d], z);
            xr[d] = scale2(om, gs_apply(di, rv[d]));
            if (d >= 1 && d <= 3) rr[d - 1] = rv[d];
        }
    };
    const int Rs = 2 * cj0 - 1, Re = 2 * cj1 - 1;
    {
        T2 rv[5], dummy[3];
        double mv[5];
        fetch_row(Rs - 1, rv, mv);
        eval_row(rv, mv, xa, dummy);
        fetch_row(Rs, rv, mv);
        eval_row(rv, mv, xb, rb);
        fetch_row(Rs + 1, rv, mv);
        eval_row(rv, mv, xq, rq);
    }
    T2 acc = zero;
    for (int R = Rs; R <= Re; ++R) {
        T2 nr[5];
        double nm[5];
        if (R < Re) fetch_row(R + 2, nr, nm);  // next row's inputs, loaded before this row is computed
        // s = r - A x1 at (c-1+k, R), k = 0..2; window rows: xa = R-1, xb = R, xq = R+1
        const double* m0 = F.mt + (long)R * sf + (c - 1);
        T2 sv[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const double* mp = m0 + k;
            MRow m;
            m.c = mp[0];
            m.e = mp[nd];
            m.w = mp[nd - 1];
            m.n = mp[2 * nd];
            m.s = mp[2 * nd - sf];
            m.ne = mp[3 * nd];
            m.sw = mp[3 * nd - sf - 1];
            T2 Ax = apply_A<T, T2>(m, nu, z, xb[k + 1], xb[k + 2], xb[k], xq[k + 1], xa[k + 1], xq[k + 2], xa[k]);
            sv[k] = sub2(rb[k], Ax);
        }
        if (R & 1) {
            if (R > Rs) {  // upper row of coarse row (R-1)/2: complete it
                acc = fma2(half, sv[1], acc);
                acc = fma2(half, sv[2], acc);
                *boff(row_of(rout, (R - 1) / 2, sc, lgST), oco) = acc;
            }
            acc = scale2(half, add2(sv[0], sv[1]));  // lower row of coarse row (R+1)/2
        } else {
            acc = fma2(half, sv[0], acc);
            acc = add2(acc, sv[1]);
            acc = fma2(half, sv[2], acc);
        }
        if (R < Re) {
#pragma unroll
            for (int d = 0; d < 5; ++d) {
                xa[d] = xb[d];
                xb[d] = xq[d];
            }
#pragma unroll
            for (int d = 0; d < 3; ++d) rb[d] = rq[d];
            eval_row(nr, nm, xq, rq);
        }
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
    const int S = sa.ST;
    for (int s = blockIdx.x * kBlock + threadIdx.x; s < S; s += gridDim.x * kBlock) {
        const GS<T> z = load_shift<T>(sa.zs, s);
        for (size_t node = 0; node < C.nodes; ++node) {
            T2 v = mk2<T>(0, 0);
            if (node == (size_t)C.side + 1) {
                T dl = (T)4 * (T)sa.nu;
                GS<T> di = gs_inv_diag<T>(dl, (T)1 / dl, (T)C.mt[node], z);
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

// Raw inputs of the pre-smoothed, coarse-corrected value x2 at one fine node: r, the
// diagonal mass entry and the (one or two) coarse values its P1 interpolation uses.
template <typename T2> struct UpIn {
    T2 r, c0, c1;
    double mc;
    int kind;  // 0: outside the grid rows, 1: coincides with a coarse node, 2: edge midpoint
};

template <typename T, typename T2>
__device__ __forceinline__ T2 up_eval(const UpIn<T2>& u, T dl, T idl, T om, const GS<T>& z) {
    if (u.kind == 0) return mk2<T>(0, 0);
    GS<T> di = gs_inv_diag<T>(dl, idl, (T)u.mc, z);
    T2 v = scale2(om, gs_apply(di, u.r));
    if (u.kind == 1) return add2(v, u.c0);
    return fma2((T)0.5, add2(u.c0, u.c1), v);
}

// x2 = omega D^{-1} r + P x_c (pre-smoothed iterate plus coarse correction), then one
// post-smoothing sweep x3 = x2 + omega D^{-1} (r - A x2). Optionally accumulates the
// dot partials of (x3, r). Each thread walks down one column: the seven x2 values of the
// stencil of row j are kept in registers and only the three new ones of row j+1,
// (i-1, j+1), (i, j+2) and (i+1, j+2), are evaluated per step; their inputs are loaded
// before the current row is computed so that the loads overlap the arithmetic.
template <typename T, bool UNI>
__global__ void __launch_bounds__(kBlock) k_vc_up(SlotArgs sa, LvArgs F, LvArgs C, const void* rin_,
                                                  const void* xc_, void* xout_, int dotmode, double* part) {
    using T2 = typename Vec2<T>::type;
    const T2* rin = (const T2*)rin_;
    const T2* xc = (const T2*)xc_;
    T2* xout = (T2*)xout_;
    const int ST = sa.ST, lgST = sa.lgST, SC = sa.slot_chunk;
    const int ls = threadIdx.x % SC, ln = threadIdx.x / SC;
    const int s = blockIdx.y * SC + ls;
    const int vb = virtual_block(sa.remap);
    const GS<T> z = load_shift<T>(sa.zs, s);
    const T nu = (T)sa.nu, om = (T)sa.omega, dl = (T)4 * nu, idl = (T)1 / dl;
    const int sf = F.side, nF = F.n, sc = C.side;
    const unsigned E = sizeof(T2);
    double acc[3] = {0, 0, 0};
    const SweepRange sr = sweep_range(vb, sa.col_groups, sa.per_step, sa.rows_per_chunk, F.side);
    int ai = sr.col0 + ln;
    if (UNI) ai = __builtin_amdgcn_readfirstlane(ai);
    if (ai > 0 && ai < nF && sr.row0 < sr.row1) {
        // per-lane byte offsets: fine columns ai-1, ai, ai+1; their coarse columns hi and hi + (bi & 1)
        unsigned ofn[3], och[3], ocq[3];
        bool odd[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int bi = ai - 1 + d, hi = bi >> 1;
            odd[d] = bi & 1;
            ofn[d] = (((unsigned)bi << lgST) + s) * E;
            och[d] = (((unsigned)hi << lgST) + s) * E;
            ocq[d] = (((unsigned)(hi + (bi & 1)) << lgST) + s) * E;
        }
        auto load = [&](int d, int bj) -> UpIn<T2> {
            UpIn<T2> u;
            if (bj < 0 || bj > nF) {
                u.kind = 0;
                u.r = u.c0 = u.c1 = mk2<T>(0, 0);
                u.mc = 0.0;
                return u;
            }
            u.r = *cboff(row_of(rin, bj, sf, lgST), ofn[d]);
            u.mc = F.mt[(long)bj * sf + ai - 1 + d];
            const int hj = bj >> 1, oj = bj & 1;
            u.c0 = *cboff(row_of(xc, hj, sc, lgST), och[d]);
            if (!odd[d] && !oj) {
                u.kind = 1;
                u.c1 = mk2<T>(0, 0);
            } else {
                u.kind = 2;
                u.c1 = *cboff(row_of(xc, hj + oj, sc, lgST), ocq[d]);
            }
            return u;
        };
        const int j0 = sr.row0;
        UpIn<T2> q0 = load(0, j0 - 1), q1 = load(1, j0 - 1), q2 = load(0, j0), q3 = load(1, j0), q4 = load(2, j0);
        UpIn<T2> q5 = load(1, j0 + 1), q6 = load(2, j0 + 1);
        T2 xsw = up_eval(q0, dl, idl, om, z), xs = up_eval(q1, dl, idl, om, z);
        T2 xw = up_eval(q2, dl, idl, om, z), xcn = up_eval(q3, dl, idl, om, z), xe = up_eval(q4, dl, idl, om, z);
        T2 xn = up_eval(q5, dl, idl, om, z), xne = up_eval(q6, dl, idl, om, z);
        T2 rc = q3.r, rn = q5.r;
        for (int aj = j0; aj < sr.row1; ++aj) {
            const bool more = aj + 1 < sr.row1;
            UpIn<T2> p0, p1, p2;
            if (more) {
                p0 = load(0, aj + 1);
                p1 = load(1, aj + 2);
                p2 = load(2, aj + 2);
            }
            T2 out = mk2<T>(0, 0);
            if (aj > 0 && aj < nF) {
                const long a = (long)aj * sf + ai;
                T2 Ax = apply_A<T, T2>(mrow(F, a), nu, z, xcn, xe, xw, xn, xs, xne, xsw);
                GS<T> da = gs_inv_diag<T>(dl, idl, (T)F.mt[a], z);
                out = add2(xcn, scale2(om, gs_apply(da, sub2(rc, Ax))));
                if (dotmode != DOT_NONE) dot3_acc(acc, out, rc, dotmode == DOT_HERM);
            }
            *boff(row_of(xout, aj, sf, lgST), ofn[1]) = out;
            if (more) {
                xsw = xw;
                xs = xcn;
                xw = up_eval(p0, dl, idl, om, z);
                xcn = xn;
                rc = rn;
                xe = xne;
                xn = up_eval(p1, dl, idl, om, z);
                rn = p1.r;
                xne = up_eval(p2, dl, idl, om, z);
            }
        }
    } else if (ai < sf) {
        const unsigned oc = (((unsigned)ai << lgST) + s) * E;
        for (int aj = sr.row0; aj < sr.row1; ++aj) *boff(row_of(xout, aj, sf, lgST), oc) = mk2<T>(0, 0);
    }
    if (dotmode != DOT_NONE) store_dot_partials(acc, part, vb, ST, blockIdx.y, SC);
}

// ---------------------------------------------------------------- operator apply

// y = A x and the dot partials of (x, A x); rolling window along the column as in k_vc_up.
template <typename T, bool UNI>
__global__ void __launch_bounds__(kBlock) k_matvec(SlotArgs sa, LvArgs F, const void* x_, void* y_, int dotmode,
                                                   double* part) {
    using T2 = typename Vec2<T>::type;
    const T2* x = (const T2*)x_;
    T2* y = (T2*)y_;
    const int ST = sa.ST, lgST = sa.lgST, SC = sa.slot_chunk;
    const int ls = threadIdx.x % SC, ln = threadIdx.x / SC;
    const int s = blockIdx.y * SC + ls;
    const int vb = virtual_block(sa.remap);
    const GS<T> z = load_shift<T>(sa.zs, s);
    const T nu = (T)sa.nu;
    const int sf = F.side, nF = F.n;
    const unsigned E = sizeof(T2);
    double acc[3] = {0, 0, 0};
    const SweepRange sr = sweep_range(vb, sa.col_groups, sa.per_step, sa.rows_per_chunk, F.side);
    int ai = sr.col0 + ln;
    if (UNI) ai = __builtin_amdgcn_readfirstlane(ai);
    if (ai > 0 && ai < nF && sr.row0 < sr.row1) {
        const unsigned ow = (((unsigned)(ai - 1) << lgST) + s) * E, oc = ow + (unsigned)ST * E,
                       oe = oc + (unsigned)ST * E;
        auto ld = [&](unsigned o, int bj) -> T2 {
            if (bj < 0 || bj > nF) return mk2<T>(0, 0);
            return *cboff(row_of(x, bj, sf, lgST), o);
        };
        const int j0 = sr.row0;
        T2 xsw = ld(ow, j0 - 1), xs = ld(oc, j0 - 1), xw = ld(ow, j0), xcn = ld(oc, j0), xe = ld(oe, j0);
        T2 xn = ld(oc, j0 + 1), xne = ld(oe, j0 + 1);
        for (int aj = j0; aj < sr.row1; ++aj) {
            const bool more = aj + 1 < sr.row1;
            T2 nw, n2, ne2;
            if (more) {  // next row's new points, loaded before this row is computed
                nw = ld(ow, aj + 1);
                n2 = ld(oc, aj + 2);
                ne2 = ld(oe, aj + 2);
            }
            T2 out = mk2<T>(0, 0);
            if (aj > 0 && aj < nF) {
                out = apply_A<T, T2>(mrow(F, (long)aj * sf + ai), nu, z, xcn, xe, xw, xn, xs, xne, xsw);
                if (dotmode != DOT_NONE) dot3_acc(acc, xcn, out, dotmode == DOT_HERM);
            }
            if (y) *boff(row_of(y, aj, sf, lgST), oc) = out;
            if (more) {
                xsw = xw;
                xs = xcn;
                xw = nw;
                xcn = xn;
                xe = xne;
                xn = n2;
                xne = ne2;
            }
        }
    } else if (ai < sf && y) {
        const unsigned oc = (((unsigned)ai << lgST) + s) * E;
        for (int aj = sr.row0; aj < sr.row1; ++aj) *boff(row_of(y, aj, sf, lgST), oc) = mk2<T>(0, 0);
    }
    if (dotmode != DOT_NONE) store_dot_partials(acc, part, vb, ST, blockIdx.y, SC);
}

// ---------------------------------------------------------------- per-slot scalars

// Sum the partials of every workgroup in a fixed order and combine them into a generic
// scalar: Hermitian u^H v = (s1 + s2) + i s3, bilinear u^T v = (s1 - s2) + i s3, and for
// slot 0 the two real dot products (s1, s2).
// Stage 1: workgroup (x, y) sums partial rows [y nblk / RB, (y+1) nblk / RB) for SG slots
// (threads: SG slots x 256/SG row lanes, lanes combined in a fixed order) into part2[y][s].
__global__ void __launch_bounds__(kBlock) k_reduce_dots1(const double* part, int nblk, int S, double* part2) {
    __shared__ double red[3][kBlock];
    const int SG = S < 64 ? S : 64, RL = kBlock / SG;
    const int sl = threadIdx.x % SG, rl = threadIdx.x / SG;
    const int s = blockIdx.x * SG + sl;
    const int RB = gridDim.y;
    const int b0 = (int)((long)blockIdx.y * nblk / RB), b1 = (int)((long)(blockIdx.y + 1) * nblk / RB);
    double s1 = 0, s2 = 0, s3 = 0;
    for (int b = b0 + rl; b < b1; b += RL) {
        const double* o = part + ((size_t)b * S + s) * 3;
        s1 += o[0];
        s2 += o[1];
        s3 += o[2];
    }
    red[0][threadIdx.x] = s1;
    red[1][threadIdx.x] = s2;
    red[2][threadIdx.x] = s3;
    __syncthreads();
    if (rl == 0) {
        for (int r = 1; r < RL; ++r) {
            s1 += red[0][r * SG + sl];
            s2 += red[1][r * SG + sl];
            s3 += red[2][r * SG + sl];
        }
        double* o = part2 + ((size_t)blockIdx.y * S + s) * 3;
        o[0] = s1;
        o[1] = s2;
        o[2] = s3;
    }
}

// Stage 2: sum the RB rows of part2 in order and combine into a generic scalar
// (S = total slots, Si = slots per instance).
__global__ void __launch_bounds__(kBlock) k_reduce_dots(const double* part, int nblk, int S, int Si, int herm,
                                                        double* out) {
    for (int s = blockIdx.x * kBlock + threadIdx.x; s < S; s += gridDim.x * kBlock) {
        double s1 = 0, s2 = 0, s3 = 0;
        for (int b = 0; b < nblk; ++b) {
            const double* o = part + ((size_t)b * S + s) * 3;
            s1 += o[0];
            s2 += o[1];
            s3 += o[2];
        }
        double2 r;
        if ((s & (Si - 1)) == 0) {
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
                                                     int Si, int* flag) {
    const double2* num = (const double2*)num_;
    const double2* den = (const double2*)den_;
    double2* coef = (double2*)coef_;
    for (int s = blockIdx.x * kBlock + threadIdx.x; s < S; s += gridDim.x * kBlock) {
        double2 a = num[s], b = den[s], r;
        if ((s & (Si - 1)) == 0) {
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
__global__ void __launch_bounds__(kBlock) k_cocg_xr(int S, int Si, size_t total, const double* coef, void* x_,
                                                    void* r_, const void* p_, const void* q_) {
    using T2 = typename Vec2<T>::type;
    T2* x = (T2*)x_;
    T2* r = (T2*)r_;
    const T2* p = (const T2*)p_;
    const T2* q = (const T2*)q_;
    for (size_t id = blockIdx.x * (size_t)kBlock + threadIdx.x; id < total; id += (size_t)gridDim.x * kBlock) {
        int s = (int)(id % S);
        GS<T> g = gs_from<T>(((const double2*)coef)[s], (s & (Si - 1)) == 0);
        x[id] = add2(x[id], gs_apply(g, p[id]));
        r[id] = sub2(r[id], gs_apply(g, q[id]));
    }
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_cocg_p(int S, int Si, size_t total, const double* coef, const void* z_,
                                                   void* p_) {
    using T2 = typename Vec2<T>::type;
    const T2* z = (const T2*)z_;
    T2* p = (T2*)p_;
    for (size_t id = blockIdx.x * (size_t)kBlock + threadIdx.x; id < total; id += (size_t)gridDim.x * kBlock) {
        int s = (int)(id % S);
        GS<T> g = gs_from<T>(((const double2*)coef)[s], (s & (Si - 1)) == 0);
        p[id] = add2(z[id], gs_apply(g, p[id]));
    }
}

// ---------------------------------------------------------------- host launchers

static SlotArgs mk_slot(const Plan& p, char* ws, const Geom& g) {
    SlotArgs sa;
    sa.S = p.S;
    sa.ST = p.ST;
    sa.lgST = 0;
    while ((1 << sa.lgST) < p.ST) ++sa.lgST;
    sa.col_groups = g.col_groups;
    sa.rows_per_chunk = g.rows_per_chunk;
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
        Geom g = slot_geom(p.lev[l + 1].side, p.ST, p.target_slot);
        SlotArgs sa = mk_slot(p, ws, g);
        dim3 grid(g.blocks, g.chunks);
        int kid = (l == 0) ? KID_DOWN0 : KID_DOWNC;
        tm_begin(p, kid, st);
        LvArgs Fl = host_lv(p, ws, l), Cl = host_lv(p, ws, l + 1);
        bool uni = g.slot_chunk >= 64;
        if (p.fp32) {
            if (uni)
                hipLaunchKernelGGL((k_vc_down<float, true>), grid, dim3(kBlock), 0, st, sa, Fl, Cl, rin, rout);
            else
                hipLaunchKernelGGL((k_vc_down<float, false>), grid, dim3(kBlock), 0, st, sa, Fl, Cl, rin, rout);
        } else {
            if (uni)
                hipLaunchKernelGGL((k_vc_down<double, true>), grid, dim3(kBlock), 0, st, sa, Fl, Cl, rin, rout);
            else
                hipLaunchKernelGGL((k_vc_down<double, false>), grid, dim3(kBlock), 0, st, sa, Fl, Cl, rin, rout);
        }
        tm_end(p, kid, st);
    }
    {
        Geom g = slot_geom(p.lev[L - 1].side, p.ST, p.target_slot);
        SlotArgs sa = mk_slot(p, ws, g);
        const void* rin = (L == 1) ? r0 : (const void*)(ws + p.lev[L - 1].off_r);
        void* xout = (L == 1) ? x0 : (void*)(ws + p.lev[L - 1].off_x);
        int grid = (p.ST + kBlock - 1) / kBlock;
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
        Geom g = slot_geom(p.lev[l].side, p.ST, p.target_slot);
        SlotArgs sa = mk_slot(p, ws, g);
        dim3 grid(g.blocks, g.chunks);
        int dm = (l == 0) ? dotmode : DOT_NONE;
        int kid = (l == 0) ? KID_UP0 : KID_UPC;
        tm_begin(p, kid, st);
        LvArgs Fl = host_lv(p, ws, l), Cl = host_lv(p, ws, l + 1);
        bool uni = g.slot_chunk >= 64;
        if (p.fp32) {
            if (uni)
                hipLaunchKernelGGL((k_vc_up<float, true>), grid, dim3(kBlock), 0, st, sa, Fl, Cl, rin, xc, xout, dm, part);
            else
                hipLaunchKernelGGL((k_vc_up<float, false>), grid, dim3(kBlock), 0, st, sa, Fl, Cl, rin, xc, xout, dm,
                                   part);
        } else {
            if (uni)
                hipLaunchKernelGGL((k_vc_up<double, true>), grid, dim3(kBlock), 0, st, sa, Fl, Cl, rin, xc, xout, dm,
                                   part);
            else
                hipLaunchKernelGGL((k_vc_up<double, false>), grid, dim3(kBlock), 0, st, sa, Fl, Cl, rin, xc, xout, dm,
                                   part);
        }
        tm_end(p, kid, st);
    }
}

void launch_matvec(const Plan& p, char* ws, const void* x, void* y, int dotmode, double* part, hipStream_t st) {
    const Geom& g = p.g_slot0;
    SlotArgs sa = mk_slot(p, ws, g);
    dim3 grid(g.blocks, g.chunks);
    LvArgs Fl = host_lv(p, ws, 0);
    bool uni = g.slot_chunk >= 64;
    if (p.fp32) {
        if (uni)
            hipLaunchKernelGGL((k_matvec<float, true>), grid, dim3(kBlock), 0, st, sa, Fl, x, y, dotmode, part);
        else
            hipLaunchKernelGGL((k_matvec<float, false>), grid, dim3(kBlock), 0, st, sa, Fl, x, y, dotmode, part);
    } else {
        if (uni)
            hipLaunchKernelGGL((k_matvec<double, true>), grid, dim3(kBlock), 0, st, sa, Fl, x, y, dotmode, part);
        else
            hipLaunchKernelGGL((k_matvec<double, false>), grid, dim3(kBlock), 0, st, sa, Fl, x, y, dotmode, part);
    }
}

void launch_reduce_dots(const Plan& p, double* part, int dotmode, double* out, hipStream_t st) {
    // stage 1 into the tail of the partial buffer, then stage 2
    const int nblk = p.g_slot0.blocks;
    const int RB = nblk < kReduceRows ? nblk : kReduceRows;
    const int SG = p.ST < 64 ? p.ST : 64;
    double* part2 = part + (size_t)nblk * p.ST * 3;
    hipLaunchKernelGGL(k_reduce_dots1, dim3((p.ST + SG - 1) / SG, RB), dim3(kBlock), 0, st, (const double*)part, nblk,
                       p.ST, part2);
    int grid = (p.ST + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_reduce_dots, dim3(grid), dim3(kBlock), 0, st, (const double*)part2, RB, p.ST, p.S,
                       dotmode == DOT_HERM ? 1 : 0, out);
}

void launch_slot_div(const Plan& p, const double* num, const double* den, double* coef, int* flag, hipStream_t st) {
    int grid = (p.ST + kBlock - 1) / kBlock;
    hipLaunchKernelGGL(k_slot_div, dim3(grid), dim3(kBlock), 0, st, num, den, coef, p.ST, p.S, flag);
}

void launch_cocg_xr(const Plan& p, const double* coef, void* x, void* r, const void* pv, const void* q,
                    hipStream_t st) {
    size_t total = p.nodes * (size_t)p.ST;
    if (p.fp32)
        hipLaunchKernelGGL(k_cocg_xr<float>, dim3(flat_grid(total)), dim3(kBlock), 0, st, p.ST, p.S, total, coef, x, r,
                           pv, q);
    else
        hipLaunchKernelGGL(k_cocg_xr<double>, dim3(flat_grid(total)), dim3(kBlock), 0, st, p.ST, p.S, total, coef, x,
                           r, pv, q);
}

void launch_cocg_p(const Plan& p, const double* coef, const void* z, void* pv, hipStream_t st) {
    size_t total = p.nodes * (size_t)p.ST;
    if (p.fp32)
        hipLaunchKernelGGL(k_cocg_p<float>, dim3(flat_grid(total)), dim3(kBlock), 0, st, p.ST, p.S, total, coef, z, pv);
    else
        hipLaunchKernelGGL(k_cocg_p<double>, dim3(flat_grid(total)), dim3(kBlock), 0, st, p.ST, p.S, total, coef, z,
                           pv);
}

// Plain 16-byte copies and fills as kernels (rather than hipMemcpyAsync / hipMemsetAsync),
// so that the outer step can be captured into a HIP graph.
__global__ void __launch_bounds__(kBlock) k_copy16(const uint4* __restrict__ src, uint4* __restrict__ dst, size_t n16) {
    for (size_t id = blockIdx.x * (size_t)kBlock + threadIdx.x; id < n16; id += (size_t)gridDim.x * kBlock)
        dst[id] = src[id];
}

__global__ void __launch_bounds__(kBlock) k_zero16(uint4* __restrict__ dst, size_t n16) {
    for (size_t id = blockIdx.x * (size_t)kBlock + threadIdx.x; id < n16; id += (size_t)gridDim.x * kBlock)
        dst[id] = make_uint4(0u, 0u, 0u, 0u);
}

void launch_copy16(const void* src, void* dst, size_t bytes, hipStream_t st) {
    size_t n16 = bytes / 16;
    hipLaunchKernelGGL(k_copy16, dim3(flat_grid(n16)), dim3(kBlock), 0, st, (const uint4*)src, (uint4*)dst, n16);
}

void launch_zero16(void* dst, size_t bytes, hipStream_t st) {
    size_t n16 = bytes / 16;
    hipLaunchKernelGGL(k_zero16, dim3(flat_grid(n16)), dim3(kBlock), 0, st, (uint4*)dst, n16);
}

void launch_copy_slots(const Plan& p, const void* src, void* dst, hipStream_t st) {
    launch_copy16(src, dst, p.nodes * (size_t)p.ST * p.elem, st);
}

}  // namespace pt
