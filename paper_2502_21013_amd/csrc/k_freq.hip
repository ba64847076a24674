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
// on the 2 x 2-cell grid (one unknown). A V(1,1) cycle (k_vc_down, k_vc_up) is symmetric
// (B^T = B, as COCG needs); a V(0,1) cycle (k_vc_restrict, k_vc_up without pre-smoothing)
// skips the pre-smoothing sweep and its operator evaluation on every level.
#include <type_traits>

#include "pt_device.h"

namespace pt {

struct LvArgs {
    int n, side;
    size_t nodes;
    const double* mt;
    const double* kt;  // Khat stencil table (per-region Khat), or null: Khat = nu_max * 5-point stencil
};

// S: slots per instance (a power of two; slot s with s % S == 0 packs k = 0 and k = N/2),
// ST = B S: slots per node over the B instances of a batch (the row stride).
struct SlotArgs {
    int S, ST, lgST, per_step, slot_chunk, remap, col_groups, rows_per_chunk;
    double nu, omega;
    const double* zs;  // S x 3 generic (a, b, c) of the shifts
};

// The levels of at most kSmallSide points per side (33, 17, 9, 5 and 3: at most kMaxSmall of
// them) run in one k_vc_small launch; r and x of level q at off_r[q], off_x[q], a scratch
// vector of the first level's size at off_t (offsets in slot values of LDS).
constexpr int kSmallSide = 33;
constexpr int kMaxSmall = 5;
struct SmallArgs {
    int count, pre;   // pre: V(1,1) (pre-smoothing), else V(0,1)
    int side[kMaxSmall];
    const double* mt[kMaxSmall];
    const double* kt[kMaxSmall];  // Khat stencil tables (per-region Khat), or null
    int off_r[kMaxSmall], off_x[kMaxSmall], off_t;
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

// Row a of a symmetric 7-point stencil table in the layout [centre | E | N | NE][nodes] (the W,
// S and SW couplings are the E, N and NE entries of the neighbours).
template <bool UNI>
__device__ __forceinline__ MRow stencil_row(const double* t, long nd, long sd, long a) {
    MRow m;
    m.c = uload<UNI>(t, a);
    m.e = uload<UNI>(t, nd + a);
    m.w = uload<UNI>(t, nd + a - 1);
    m.n = uload<UNI>(t, 2 * nd + a);
    m.s = uload<UNI>(t, 2 * nd + a - sd);
    m.ne = uload<UNI>(t, 3 * nd + a);
    m.sw = uload<UNI>(t, 3 * nd + a - sd - 1);
    return m;
}

template <bool UNI>
__device__ __forceinline__ MRow mrow(const LvArgs& L, long a) {
    return stencil_row<UNI>(L.mt, (long)L.nodes, (long)L.side, a);
}

// the Khat row of node a (per-region Khat; the same layout as the mass)
template <bool UNI>
__device__ __forceinline__ MRow krow(const LvArgs& L, long a) {
    return stencil_row<UNI>(L.kt, (long)L.nodes, (long)L.side, a);
}

// V consecutive slots of one node held by one lane: V = 2 in FP32 mode (one 16-byte
// access), V = 1 in FP64 mode (a double2). Slot vectors are read and written in these
// units, which halves the memory instructions of the FP32 sweeps.
template <typename T> struct LaneW;
template <> struct LaneW<float> { static constexpr int V = 2; };
template <> struct LaneW<double> { static constexpr int V = 1; };

template <typename T> struct alignas(16) SV {
    static constexpr int V = LaneW<T>::V;
    typename Vec2<T>::type v[V];
};

template <typename T> __device__ __forceinline__ SV<T> sv_zero() {
    SV<T> r;
#pragma unroll
    for (int k = 0; k < SV<T>::V; ++k) r.v[k] = mk2<T>(0, 0);
    return r;
}
template <typename T> __device__ __forceinline__ SV<T> sv_add(const SV<T>& a, const SV<T>& b) {
    SV<T> r;
#pragma unroll
    for (int k = 0; k < SV<T>::V; ++k) r.v[k] = add2(a.v[k], b.v[k]);
    return r;
}
template <typename T> __device__ __forceinline__ SV<T> sv_sub(const SV<T>& a, const SV<T>& b) {
    SV<T> r;
#pragma unroll
    for (int k = 0; k < SV<T>::V; ++k) r.v[k] = sub2(a.v[k], b.v[k]);
    return r;
}
template <typename T> __device__ __forceinline__ SV<T> sv_scale(T s, const SV<T>& a) {
    SV<T> r;
#pragma unroll
    for (int k = 0; k < SV<T>::V; ++k) r.v[k] = scale2(s, a.v[k]);
    return r;
}
// acc + s a
template <typename T> __device__ __forceinline__ SV<T> sv_fma(T s, const SV<T>& a, const SV<T>& acc) {
    SV<T> r;
#pragma unroll
    for (int k = 0; k < SV<T>::V; ++k) r.v[k] = fma2(s, a.v[k], acc.v[k]);
    return r;
}

// (A x)_a for interior node a with mass row m, given the 7 neighbour values of x; z[k] is
// the shift of the lane's slot k. MASS = false: the mass row is zero (stiffness part only);
// MASS = true: the mass part is added without a branch (no change where the row is zero).
// VK = false: Khat = nu * (5-point stencil); VK = true: Khat from the stencil row kr.
template <typename T, bool MASS, bool VK = false>
__device__ __forceinline__ SV<T> apply_A_t(const MRow& m, T nu, const GS<T>* z, const SV<T>& xc, const SV<T>& xe,
                                           const SV<T>& xw, const SV<T>& xn, const SV<T>& xs, const SV<T>& xne,
                                           const SV<T>& xsw, const MRow& kr = MRow{}) {
    SV<T> out;
    if constexpr (VK) {
        const T kc = (T)kr.c, ke = (T)kr.e, kw = (T)kr.w, kn = (T)kr.n, ks = (T)kr.s, kne = (T)kr.ne, ksw = (T)kr.sw;
#pragma unroll
        for (int k = 0; k < SV<T>::V; ++k) {
            auto Kx = scale2(kc, xc.v[k]);
            Kx = fma2(ke, xe.v[k], Kx);
            Kx = fma2(kw, xw.v[k], Kx);
            Kx = fma2(kn, xn.v[k], Kx);
            Kx = fma2(ks, xs.v[k], Kx);
            Kx = fma2(kne, xne.v[k], Kx);
            out.v[k] = fma2(ksw, xsw.v[k], Kx);
        }
    } else {
#pragma unroll
        for (int k = 0; k < SV<T>::V; ++k) {
            out.v[k].x = nu * ((T)4 * xc.v[k].x - xe.v[k].x - xw.v[k].x - xn.v[k].x - xs.v[k].x);
            out.v[k].y = nu * ((T)4 * xc.v[k].y - xe.v[k].y - xw.v[k].y - xn.v[k].y - xs.v[k].y);
        }
    }
    if constexpr (!MASS) return out;
    const T mc = (T)m.c, me = (T)m.e, mw = (T)m.w, mn = (T)m.n, ms = (T)m.s, mne = (T)m.ne, msw = (T)m.sw;
#pragma unroll
    for (int k = 0; k < SV<T>::V; ++k) {
        auto Mx = scale2(mc, xc.v[k]);
        Mx = fma2(me, xe.v[k], Mx);
        Mx = fma2(mw, xw.v[k], Mx);
        Mx = fma2(mn, xn.v[k], Mx);
        Mx = fma2(ms, xs.v[k], Mx);
        Mx = fma2(mne, xne.v[k], Mx);
        Mx = fma2(msw, xsw.v[k], Mx);
        out.v[k] = add2(out.v[k], gs_apply(z[k], Mx));
    }
    return out;
}

template <typename T, bool VK = false>
__device__ __forceinline__ SV<T> apply_A(const MRow& m, T nu, const GS<T>* z, const SV<T>& xc, const SV<T>& xe,
                                         const SV<T>& xw, const SV<T>& xn, const SV<T>& xs, const SV<T>& xne,
                                         const SV<T>& xsw, const MRow& kr = MRow{}) {
    if (m.any()) return apply_A_t<T, true, VK>(m, nu, z, xc, xe, xw, xn, xs, xne, xsw, kr);
    return apply_A_t<T, false, VK>(m, nu, z, xc, xe, xw, xn, xs, xne, xsw, kr);
}

// omega D^{-1} r with D = dl + z diag(M) (dm the node's diagonal mass entry). MASS = false:
// dm = 0; MASS = true: any dm, the inverse chosen without a branch (same values as gs_inv_diag).
template <typename T, bool MASS>
__device__ __forceinline__ SV<T> jacobi_t(T dl, T idl, T om, double dm, const GS<T>* z, const SV<T>& r) {
    SV<T> out;
    if constexpr (!MASS) {
        // D = dl: a real scaling (omega / dl per component)
        const T s = om * idl;
#pragma unroll
        for (int k = 0; k < SV<T>::V; ++k) out.v[k] = scale2(s, r.v[k]);
        return out;
    }
#pragma unroll
    for (int k = 0; k < SV<T>::V; ++k) {
        const GS<T> di = gs_inv_diag_sel<T>(dl, idl, (T)dm, z[k]);
        out.v[k] = scale2(om, gs_apply(di, r.v[k]));
    }
    return out;
}

template <typename T> __device__ __forceinline__ void sv_dot_acc(double (*acc)[3], const SV<T>& u, const SV<T>& v,
                                                                bool conj) {
#pragma unroll
    for (int k = 0; k < SV<T>::V; ++k) dot3_acc(acc[k], u.v[k], v.v[k], conj);
}

// Lane geometry of the slot-vector kernels: a workgroup row of SC lanes covers SC V
// consecutive slots; lane ls of slot chunk blockIdx.y starts at slot s0.
template <typename T> struct SlotLane {
    int ls, ln, s0;
    GS<T> z[SV<T>::V];
};

template <typename T> __device__ __forceinline__ SlotLane<T> slot_lane(const SlotArgs& sa) {
    SlotLane<T> L;
    constexpr int V = SV<T>::V;
    L.ls = threadIdx.x % sa.slot_chunk;
    L.ln = threadIdx.x / sa.slot_chunk;
    L.s0 = (blockIdx.y * sa.slot_chunk + L.ls) * V;
#pragma unroll
    for (int k = 0; k < V; ++k) L.z[k] = load_shift<T>(sa.zs, L.s0 + k);
    return L;
}

// ---------------------------------------------------------------- dot-product partials

// Reduce the per-thread partial sums of a workgroup over threads sharing a slot and
// store them at part[(vb * ST + s) * 3 + c].
template <int V>
__device__ __forceinline__ void store_dot_partials(const double (*acc)[3], double* part, int vb, int ST, int chunk,
                                                   int SC) {
    __shared__ double red[3][kBlock * V];
#pragma unroll
    for (int k = 0; k < V; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) red[c][threadIdx.x * V + k] = acc[k][c];
    __syncthreads();
    const int SL = SC * V;  // slots per workgroup row
    for (int q = threadIdx.x; q < SL; q += kBlock) {
        double s0 = 0, s1 = 0, s2 = 0;
        for (int t = q; t < kBlock * V; t += SL) {
            s0 += red[0][t];
            s1 += red[1][t];
            s2 += red[2][t];
        }
        const size_t s = (size_t)chunk * SL + q;
        double* o = part + ((size_t)vb * ST + s) * 3;
        o[0] = s0;
        o[1] = s1;
        o[2] = s2;
    }
}

// ---------------------------------------------------------------- V-cycle: down

// r_c = P^T (r - A x1) with the pre-smoothed x1 = omega D^{-1} r (one Jacobi sweep from
// zero). Thread (coarse column ci, slots) walks up the fine rows R around fine column
// c = 2 ci with a 3-row x 5-column register window of x1 (rows R-1..R+1, columns
// c-2..c+2), forms the fine residual s = r - A x1 at columns c-1, c, c+1 of row R and adds
// it into the coarse rows it belongs to with the P^T weights: row 2cj-1 contributes
// (c-1, c) x 1/2, row 2cj contributes (c-1, c, c+1) x (1/2, 1, 1/2), row 2cj+1
// contributes (c, c+1) x 1/2 (P1 interpolation on the SW-NE split grid). The inputs of
// row R+2 are loaded before row R is computed, on every path (the row clamped to the grid
// after the last one), and the mass rows of a uniform column come through the scalar unit,
// so that the wait for a row's inputs never waits for the loads of the row after it. The
// coarse residual is stored with streaming access (it is read back only by the next level).
template <typename T, bool UNI, bool VK>
__global__ void __launch_bounds__(kBlock) k_vc_down(SlotArgs sa, LvArgs F, LvArgs C, const void* rin_, void* rout_) {
    using W = SV<T>;
    const W* rin = (const W*)rin_;
    W* rout = (W*)rout_;
    const int lgST = sa.lgST;
    const SlotLane<T> L = slot_lane<T>(sa);
    const int vb = virtual_block(sa.remap);
    const T nu = (T)sa.nu, om = (T)sa.omega, dl = (T)4 * nu, idl = (T)1 / dl;
    const int sf = F.side, nF = F.n, sc = C.side, nc = C.n;
    const long nd = (long)F.nodes;
    const T half = (T)0.5;
    const unsigned E = sizeof(typename Vec2<T>::type);
    const SweepRange sr = sweep_range(vb, sa.col_groups, sa.per_step, sa.rows_per_chunk, sc);
    int ci = sr.col0 + L.ln;
    if (UNI) ci = __builtin_amdgcn_readfirstlane(ci);
    if (ci >= sc) return;
    const W zero = sv_zero<T>();
    const unsigned oco = (((unsigned)ci << lgST) + L.s0) * E;
    // boundary coarse nodes of this chunk are zero
    for (int cj = sr.row0; cj < sr.row1; ++cj)
        if (ci == 0 || ci == nc || cj == 0 || cj == nc) *boff(row_of(rout, cj, sc, lgST - (W::V - 1)), oco) = zero;
    if (ci == 0 || ci == nc) return;
    const int cj0 = sr.row0 > 1 ? sr.row0 : 1;
    const int cj1 = sr.row1 < nc ? sr.row1 : nc;  // interior coarse rows [cj0, cj1)
    if (cj0 >= cj1) return;
    const int c = 2 * ci;
    const int lgR = lgST - (W::V - 1);  // row stride in lane units: 2^lgST slots = 2^lgR units
    unsigned of[5];
#pragma unroll
    for (int d = 0; d < 5; ++d) of[d] = (((unsigned)(c - 2 + d) << lgST) + L.s0) * E;
    // rows 2 cj0 - 2 .. 2 cj1 (all inside the grid, 0 <= R <= nF) are fetched
    // mv[d]: diagonal mass of column c-2+d; mv[5+d]: its Khat diagonal (VK)
    auto fetch_row = [&](int R, W* rv, double* mv) {
        const W* fr = row_of(rin, R, sf, lgR);
        const long mr = (long)R * sf + (c - 2);
#pragma unroll
        for (int d = 0; d < 5; ++d) {
            rv[d] = *cboff(fr, of[d]);
            mv[d] = uload<UNI>(F.mt, mr + d);
            if constexpr (VK) mv[5 + d] = uload<UNI>(F.kt, mr + d);
        }
    };
    // x1 on a row: one branch per row (uniform) on whether any of its five diagonal mass
    // entries is nonzero, then five independent Jacobi steps
    auto eval_row = [&](const W* rv, const double* mv, W* xr, W* rr) {
        T dd[5], idd[5];
#pragma unroll
        for (int d = 0; d < 5; ++d) {
            dd[d] = VK ? (T)mv[5 + d] : dl;
            idd[d] = VK ? (T)1 / dd[d] : idl;
        }
        const bool anym = mv[0] != 0.0 || mv[1] != 0.0 || mv[2] != 0.0 || mv[3] != 0.0 || mv[4] != 0.0;
        if (anym) {
#pragma unroll
            for (int d = 0; d < 5; ++d) xr[d] = jacobi_t<T, true>(dd[d], idd[d], om, mv[d], L.z, rv[d]);
        } else {
#pragma unroll
            for (int d = 0; d < 5; ++d) xr[d] = jacobi_t<T, false>(dd[d], idd[d], om, mv[d], L.z, rv[d]);
        }
#pragma unroll
        for (int d = 1; d <= 3; ++d) rr[d - 1] = rv[d];
    };
    const int Rs = 2 * cj0 - 1, Re = 2 * cj1 - 1;
    // x1 on rows R-1, R, R+1 and r on rows R, R+1 in rings over the row (row t in slot
    // (t - Rs + 1) mod 3), the row loop unrolled by 3 so that no value is moved
    W X[3][5], Rr[3][3];
    {
        W rv[5];
        double mv[10];
        fetch_row(Rs - 1, rv, mv);
        eval_row(rv, mv, X[0], Rr[0]);
        fetch_row(Rs, rv, mv);
        eval_row(rv, mv, X[1], Rr[1]);
        fetch_row(Rs + 1, rv, mv);
        eval_row(rv, mv, X[2], Rr[2]);
    }
    W acc = zero;
    auto step = [&](int R, auto u_) {
        constexpr int u = decltype(u_)::value;  // (R - Rs) mod 3
        constexpr int ia = u, ib = (u + 1) % 3, iq = (u + 2) % 3;
        W nr[5];
        double nm[10];
        // next row's inputs, loaded before this row is computed (unused after the last row)
        fetch_row(R + 2 < nF ? R + 2 : nF, nr, nm);
        issue_fence();
        if (R > Re) return;
        const W* xa = X[ia];
        const W* xb = X[ib];
        const W* xq = X[iq];
        const W* rb = Rr[ib];
        // s = r - A x1 at (c-1+k, R), k = 0..2; rows: xa = R-1, xb = R, xq = R+1
        const long m0 = (long)R * sf + (c - 1);
        W sv[3];
        MRow mr3[3], kr3[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            mr3[k] = mrow<UNI>(F, m0 + k);
            if constexpr (VK) kr3[k] = krow<UNI>(F, m0 + k);
        }
        // one branch per row on whether any of the three mass rows is nonzero
        if (mr3[0].any() || mr3[1].any() || mr3[2].any()) {
#pragma unroll
            for (int k = 0; k < 3; ++k)
                sv[k] = sv_sub(rb[k], apply_A_t<T, true, VK>(mr3[k], nu, L.z, xb[k + 1], xb[k + 2], xb[k], xq[k + 1],
                                                             xa[k + 1], xq[k + 2], xa[k], kr3[k]));
        } else {
#pragma unroll
            for (int k = 0; k < 3; ++k)
                sv[k] = sv_sub(rb[k], apply_A_t<T, false, VK>(mr3[k], nu, L.z, xb[k + 1], xb[k + 2], xb[k], xq[k + 1],
                                                              xa[k + 1], xq[k + 2], xa[k], kr3[k]));
        }
        if (R & 1) {
            if (R > Rs) {  // upper row of coarse row (R-1)/2: complete it
                acc = sv_fma(half, sv[1], acc);
                acc = sv_fma(half, sv[2], acc);
                nt_store(boff(row_of(rout, (R - 1) / 2, sc, lgR), oco), acc);
            }
            acc = sv_scale(half, sv_add(sv[0], sv[1]));  // lower row of coarse row (R+1)/2
        } else {
            acc = sv_fma(half, sv[0], acc);
            acc = sv_add(acc, sv[1]);
            acc = sv_fma(half, sv[2], acc);
        }
        if (R < Re) eval_row(nr, nm, X[ia], Rr[ia]);  // row R+2 over row R-1
    };
    for (int R = Rs; R <= Re; R += 3) {
        step(R, std::integral_constant<int, 0>());
        step(R + 1, std::integral_constant<int, 1>());
        step(R + 2, std::integral_constant<int, 2>());
    }
}

// ---------------------------------------------------------------- V(0,1) cycle: restriction

// r_c = P^T r, the restriction of the V(0,1) cycle (no pre-smoothing, so the fine residual is r
// itself; r is zero on the boundary). Thread (coarse column ci, slots) walks the coarse rows of
// its chunk with the P^T weights of k_vc_down: fine row 2cj contributes (c-1, c, c+1) x
// (1/2, 1, 1/2), row 2cj+1 contributes (c, c+1) x 1/2 to coarse row cj and (c-1, c) x 1/2 to
// coarse row cj+1 (carried), so each fine row is loaded once per walk (three columns). The two
// fine rows of the next coarse row are loaded before the current one is computed, on every path
// (rows clamped to the grid past the last one). Little arithmetic: the sweep streams r.
template <typename T, bool UNI>
__global__ void __launch_bounds__(kBlock) k_vc_restrict(SlotArgs sa, LvArgs F, LvArgs C, const void* rin_,
                                                        void* rout_) {
    using W = SV<T>;
    const W* rin = (const W*)rin_;
    W* rout = (W*)rout_;
    const int lgST = sa.lgST, lgR = lgST - (W::V - 1);
    const SlotLane<T> L = slot_lane<T>(sa);
    const int vb = virtual_block(sa.remap);
    const int sf = F.side, nF = F.n, sc = C.side, nc = C.n;
    const T half = (T)0.5;
    const unsigned E = sizeof(typename Vec2<T>::type);
    const SweepRange sr = sweep_range(vb, sa.col_groups, sa.per_step, sa.rows_per_chunk, sc);
    int ci = sr.col0 + L.ln;
    if (UNI) ci = __builtin_amdgcn_readfirstlane(ci);
    if (ci >= sc || sr.row0 >= sr.row1) return;
    const W zero = sv_zero<T>();
    const unsigned oco = (((unsigned)ci << lgST) + L.s0) * E;
    if (ci == 0 || ci == nc) {
        for (int cj = sr.row0; cj < sr.row1; ++cj) nt_store(boff(row_of(rout, cj, sc, lgR), oco), zero);
        return;
    }
    const int c = 2 * ci;
    unsigned of[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) of[d] = (((unsigned)(c - 1 + d) << lgST) + L.s0) * E;
    // fine rows 2 cj and 2 cj + 1 (clamped onto the grid) at columns c-1, c, c+1
    auto fetch = [&](int cj, W* a, W* b) {
        const W* ra = row_of(rin, clampi(2 * cj, 0, nF), sf, lgR);
        const W* rb = row_of(rin, clampi(2 * cj + 1, 0, nF), sf, lgR);
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            a[d] = *cboff(ra, of[d]);
            b[d] = *cboff(rb, of[d]);
        }
    };
    // (c-1, c) x 1/2 of fine row 2 row0 - 1 (the part of the first coarse row from below)
    W carry = zero;
    if (sr.row0 > 0) {
        const W* rp = row_of(rin, 2 * sr.row0 - 1, sf, lgR);
        carry = sv_scale(half, sv_add(*cboff(rp, of[0]), *cboff(rp, of[1])));
    }
    W A0[3], B0[3], A1[3], B1[3];
    fetch(sr.row0, A0, B0);
    auto step = [&](int cj, W* a, W* b, W* na, W* nb) {
        fetch(cj + 1, na, nb);
        issue_fence();
        W acc = zero;
        if (cj > 0 && cj < nc) {
            acc = sv_fma(half, a[0], carry);
            acc = sv_add(acc, a[1]);
            acc = sv_fma(half, a[2], acc);
            acc = sv_fma(half, b[1], acc);
            acc = sv_fma(half, b[2], acc);
        }
        nt_store(boff(row_of(rout, cj, sc, lgR), oco), acc);
        carry = sv_scale(half, sv_add(b[0], b[1]));
    };
    int cj = sr.row0;
    for (; cj + 1 < sr.row1; cj += 2) {
        step(cj, A0, B0, A1, B1);
        step(cj + 1, A1, B1, A0, B0);
    }
    if (cj < sr.row1) step(cj, A0, B0, A1, B1);
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
                T dl = C.kt ? (T)C.kt[node] : (T)4 * (T)sa.nu;   // Khat's diagonal
                GS<T> di = gs_inv_diag<T>(dl, (T)1 / dl, (T)C.mt[node], z);
                v = gs_apply(di, rin[node * S + s]);
            }
            xout[node * S + s] = v;
        }
    }
}

// ---------------------------------------------------------------- V-cycle: small levels

// The levels from l0 (side <= kSmallSide, l0 >= 1) to the coarsest in one launch. Workgroup s
// takes slot s, keeps r and x of all these levels in LDS and runs the same V(1,1) cycle as
// k_vc_down, k_vc_coarsest and k_vc_up: restriction of r - A x1 with x1 = omega D^{-1} r, the
// exact solve on the 2 x 2-cell grid, then x2 = omega D^{-1} r + P x_c and
// x3 = x2 + omega D^{-1} (r - A x2), phases separated by workgroup barriers (sm.pre = 0: the
// V(0,1) cycle of k_vc_restrict and k_vc_up, x1 = 0 and x2 = P x_c). As separate
// launches these levels cost a few microseconds each for very little work.
template <typename T>
__global__ void __launch_bounds__(kBlock) k_vc_small(SlotArgs sa, SmallArgs sm, const void* rin_, void* xout_) {
    using T2 = typename Vec2<T>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T2* sh = (T2*)smem_raw;
    const T2* rin = (const T2*)rin_;
    T2* xout = (T2*)xout_;
    const int ST = sa.ST, s = blockIdx.x;
    const GS<T> z = load_shift<T>(sa.zs, s);
    const T nu = (T)sa.nu, om = (T)sa.omega, dl = (T)4 * nu, idl = (T)1 / dl, half = (T)0.5;
    const T2 zero = mk2<T>(0, 0);
    // omega D^{-1} v at node a of a level with mass table mt and Khat table kt (null: Khat = nu_max
    // times the 5-point stencil), D = Khat_aa + z M_aa (the forms of jacobi_t)
    auto jac = [&](const double* mt, const double* kt, int a, T2 v) -> T2 {
        const double dm = mt[a];
        const T dla = kt ? (T)kt[a] : dl, idla = kt ? (T)1 / dla : idl;
        if (dm == 0.0) return scale2(om * idla, v);
        return scale2(om, gs_apply(gs_inv_diag_sel<T>(dla, idla, (T)dm, z), v));
    };
    // (A x)_a at interior node a of a level with side sd and tables mt, kt (as apply_A_t)
    auto applyA = [&](const double* mt, const double* kt, int sd, const T2* xv, int a) -> T2 {
        const int nd = sd * sd;
        const T2 xc = xv[a], xe = xv[a + 1], xw = xv[a - 1], xn = xv[a + sd], xs = xv[a - sd], xne = xv[a + sd + 1],
                 xsw = xv[a - sd - 1];
        T2 out;
        if (kt) {
            out = scale2((T)kt[a], xc);
            out = fma2((T)kt[nd + a], xe, out);
            out = fma2((T)kt[nd + a - 1], xw, out);
            out = fma2((T)kt[2 * nd + a], xn, out);
            out = fma2((T)kt[2 * nd + a - sd], xs, out);
            out = fma2((T)kt[3 * nd + a], xne, out);
            out = fma2((T)kt[3 * nd + a - sd - 1], xsw, out);
        } else {
            out.x = nu * ((T)4 * xc.x - xe.x - xw.x - xn.x - xs.x);
            out.y = nu * ((T)4 * xc.y - xe.y - xw.y - xn.y - xs.y);
        }
        const double mc = mt[a], me = mt[nd + a], mw = mt[nd + a - 1], mn = mt[2 * nd + a], ms = mt[2 * nd + a - sd],
                     mne = mt[3 * nd + a], msw = mt[3 * nd + a - sd - 1];
        if (mc != 0.0 || me != 0.0 || mw != 0.0 || mn != 0.0 || ms != 0.0 || mne != 0.0 || msw != 0.0) {
            T2 Mx = scale2((T)mc, xc);
            Mx = fma2((T)me, xe, Mx);
            Mx = fma2((T)mw, xw, Mx);
            Mx = fma2((T)mn, xn, Mx);
            Mx = fma2((T)ms, xs, Mx);
            Mx = fma2((T)mne, xne, Mx);
            Mx = fma2((T)msw, xsw, Mx);
            out = add2(out, gs_apply(z, Mx));
        }
        return out;
    };
    {
        const int nodes = sm.side[0] * sm.side[0];
        T2* r = sh + sm.off_r[0];
        for (int a = threadIdx.x; a < nodes; a += kBlock) r[a] = rin[(size_t)a * ST + s];
    }
    __syncthreads();
    // restriction sweeps: level q -> q + 1
    for (int q = 0; q + 1 < sm.count; ++q) {
        const int sd = sm.side[q], n = sd - 1, nodes = sd * sd, sc = sm.side[q + 1], nc = sc - 1;
        const double* mt = sm.mt[q];
        const double* kt = sm.kt[q];
        const T2* r = sh + sm.off_r[q];
        T2* x1 = sh + sm.off_x[q];
        const T2* t = r;   // the fine residual (V(0,1): r itself)
        if (sm.pre) {
            T2* tw = sh + sm.off_t;
            for (int a = threadIdx.x; a < nodes; a += kBlock) x1[a] = jac(mt, kt, a, r[a]);
            __syncthreads();
            for (int a = threadIdx.x; a < nodes; a += kBlock) {
                const int j = a / sd, i = a - j * sd;
                tw[a] = (i > 0 && i < n && j > 0 && j < n) ? sub2(r[a], applyA(mt, kt, sd, x1, a)) : zero;
            }
            __syncthreads();
            t = tw;
        }
        T2* rc = sh + sm.off_r[q + 1];
        for (int ca = threadIdx.x; ca < sc * sc; ca += kBlock) {
            const int cj = ca / sc, ci = ca - cj * sc;
            T2 acc = zero;
            if (ci > 0 && ci < nc && cj > 0 && cj < nc) {
                // P^T at fine node (2 ci, 2 cj): W, C, E of its row, (C, E) above, (W, C) below
                const int a = 2 * cj * sd + 2 * ci;
                acc = scale2(half, add2(t[a - sd - 1], t[a - sd]));
                acc = fma2(half, t[a - 1], acc);
                acc = add2(acc, t[a]);
                acc = fma2(half, t[a + 1], acc);
                acc = fma2(half, t[a + sd], acc);
                acc = fma2(half, t[a + sd + 1], acc);
            }
            rc[ca] = acc;
        }
        __syncthreads();
    }
    {
        // the coarsest level: the single interior node (1, 1), 1 x 1 operator Khat_c + z M_c
        // (Khat_c = 4 nu_max for the constant stencil)
        const int q = sm.count - 1, sd = sm.side[q], nodes = sd * sd;
        const T2* r = sh + sm.off_r[q];
        T2* x = sh + sm.off_x[q];
        const T dlq = sm.kt[q] ? (T)sm.kt[q][sd + 1] : dl;
        for (int a = threadIdx.x; a < nodes; a += kBlock)
            x[a] = (a == sd + 1) ? gs_apply(gs_inv_diag<T>(dlq, (T)1 / dlq, (T)sm.mt[q][a], z), r[a]) : zero;
    }
    __syncthreads();
    // prolongation sweeps with post-smoothing: level q + 1 -> q
    for (int q = sm.count - 2; q >= 0; --q) {
        const int sd = sm.side[q], n = sd - 1, nodes = sd * sd, sc = sm.side[q + 1];
        const double* mt = sm.mt[q];
        const double* kt = sm.kt[q];
        const T2* r = sh + sm.off_r[q];
        const T2* xc = sh + sm.off_x[q + 1];
        T2* x2 = sh + sm.off_t;
        T2* x3 = sh + sm.off_x[q];
        for (int a = threadIdx.x; a < nodes; a += kBlock) {
            const int j = a / sd, i = a - j * sd, hi = i >> 1, hj = j >> 1;
            const T2 c0 = xc[hj * sc + hi];
            const T2 p = ((i | j) & 1) ? scale2(half, add2(c0, xc[(hj + (j & 1)) * sc + hi + (i & 1)])) : c0;
            x2[a] = sm.pre ? add2(jac(mt, kt, a, r[a]), p) : p;
        }
        __syncthreads();
        for (int a = threadIdx.x; a < nodes; a += kBlock) {
            const int j = a / sd, i = a - j * sd;
            x3[a] = (i > 0 && i < n && j > 0 && j < n)
                        ? add2(x2[a], jac(mt, kt, a, sub2(r[a], applyA(mt, kt, sd, x2, a))))
                        : zero;
        }
        __syncthreads();
    }
    {
        const int nodes = sm.side[0] * sm.side[0];
        const T2* x = sh + sm.off_x[0];
        for (int a = threadIdx.x; a < nodes; a += kBlock) xout[(size_t)a * ST + s] = x[a];
    }
}

// ---------------------------------------------------------------- V-cycle: up

// Raw inputs of the pre-smoothed, coarse-corrected value x2 at one fine node: r, the
// diagonal mass entry and the (one or two) coarse values its P1 interpolation uses.
template <typename W> struct UpIn {
    W r, c0, c1;
    double mc, kc;  // diagonal mass and (per-region Khat) Khat diagonal
    int kind;  // 0: outside the grid rows, 1: coincides with a coarse node, 2: edge midpoint
};

// x2 at one fine point (the kind is uniform in a column walk); MASS as in jacobi_t; PRE: the
// pre-smoothed omega D^{-1} r is part of x2 (V(1,1)), otherwise x2 = P x_c (V(0,1)); VK: D's
// Khat part is the point's own Khat diagonal
template <typename T, bool MASS, bool PRE, bool VK = false>
__device__ __forceinline__ SV<T> up_eval_t(const UpIn<SV<T>>& u, T dl, T idl, T om, const GS<T>* z) {
    if (u.kind == 0) return sv_zero<T>();
    const T dlu = VK ? (T)u.kc : dl, idlu = VK ? (T)1 / dlu : idl;
    const SV<T> v = PRE ? jacobi_t<T, MASS>(dlu, idlu, om, u.mc, z, u.r) : sv_zero<T>();
    if (u.kind == 1) return sv_add(v, u.c0);
    return sv_fma((T)0.5, sv_add(u.c0, u.c1), v);
}

// x3 = x2 + omega D^{-1} (r - A x2) at an interior node with mass row m (m.c its diagonal) and,
// VK, Khat row kr (dl = kr.c then)
template <typename T, bool MASS, bool VK = false>
__device__ __forceinline__ SV<T> post_smooth_t(const MRow& m, T nu, T dl, T idl, T om, const GS<T>* z, const SV<T>& r,
                                               const SV<T>& xc, const SV<T>& xe, const SV<T>& xw, const SV<T>& xn,
                                               const SV<T>& xs, const SV<T>& xne, const SV<T>& xsw,
                                               const MRow& kr = MRow{}) {
    const SV<T> Ax = apply_A_t<T, MASS, VK>(m, nu, z, xc, xe, xw, xn, xs, xne, xsw, kr);
    return sv_add(xc, jacobi_t<T, MASS>(dl, idl, om, m.c, z, sv_sub(r, Ax)));
}

// x2 = omega D^{-1} r + P x_c (pre-smoothed iterate plus coarse correction; PRE = false, the
// V(0,1) cycle: x2 = P x_c, and r is read on the centre column only), then one
// post-smoothing sweep x3 = x2 + omega D^{-1} (r - A x2). Optionally accumulates the
// dot partials of (x3, r). Each thread walks down one column: the seven x2 values of the
// stencil of row j are kept in registers and only the three new ones of row j+1,
// (i-1, j+1), (i, j+2) and (i+1, j+2), are evaluated per step; their inputs are loaded
// before the current row is computed so that the loads overlap the arithmetic, and the
// coarse values they interpolate from come from a window of coarse rows (below).
// Three waves per SIMD (at most 168 VGPRs): the coarse window would otherwise drop to two.
// x3 is stored with streaming access, keeping the caches for the neighbour columns' inputs.
template <typename T, bool UNI, bool PRE, bool VK>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) k_vc_up(SlotArgs sa, LvArgs F, LvArgs C, const void* rin_,
                                                  const void* xc_, void* xout_, int dotmode, double* part) {
using W = SV<T>;
    constexpr int V = W::V;
    const W* rin = (const W*)rin_;
    const W* xc = (const W*)xc_;
    W* xout = (W*)xout_;
    const int ST = sa.ST, lgST = sa.lgST, lgR = lgST - (V - 1), SC = sa.slot_chunk;
    const SlotLane<T> L = slot_lane<T>(sa);
    const int vb = virtual_block(sa.remap);
    const T nu = (T)sa.nu, om = (T)sa.omega, dl = (T)4 * nu, idl = (T)1 / dl;
    const int sf = F.side, nF = F.n, sc = C.side;
    const unsigned E = sizeof(typename Vec2<T>::type);
    double acc[V][3] = {};
    const SweepRange sr = sweep_range(vb, sa.col_groups, sa.per_step, sa.rows_per_chunk, F.side);
    int ai = sr.col0 + L.ln;
    if (UNI) ai = __builtin_amdgcn_readfirstlane(ai);
    if (ai > 0 && ai < nF && sr.row0 < sr.row1) {
        // per-lane byte offsets: fine columns ai-1, ai, ai+1; their coarse columns hi and hi + (bi & 1)
        unsigned ofn[3], och[3], ocq[3];
        bool odd[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const int bi = ai - 1 + d, hi = bi >> 1;
            odd[d] = bi & 1;
            ofn[d] = (((unsigned)bi << lgST) + L.s0) * E;
            och[d] = (((unsigned)hi << lgST) + L.s0) * E;
            ocq[d] = (((unsigned)(hi + (bi & 1)) << lgST) + L.s0) * E;
        }
        // inputs of fine point (ai-1+d, bj) for the first rows of the walk; every load is issued
        // on every path (row clamped to the grid; c1 is the node of c0 again where the point
        // coincides with a coarse node)
        auto load = [&](int d, int bj) -> UpIn<W> {
            UpIn<W> u;
            const int bc = clampi(bj, 0, nF);
            u.r = (PRE || d == 1) ? *cboff(row_of(rin, bc, sf, lgR), ofn[d]) : sv_zero<T>();
            u.mc = PRE ? uload<UNI>(F.mt, (long)bc * sf + ai - 1 + d) : 0.0;
            u.kc = (PRE && VK) ? uload<UNI>(F.kt, (long)bc * sf + ai - 1 + d) : 0.0;
            const int hj = bc >> 1, oj = bc & 1;
            u.c0 = *cboff(row_of(xc, hj, sc, lgR), och[d]);
            u.c1 = *cboff(row_of(xc, hj + oj, sc, lgR), ocq[d]);
            u.kind = (bj < 0 || bj > nF) ? 0 : ((!odd[d] && !oj) ? 1 : 2);
            return u;
        };
        const int j0 = sr.row0;
        W xsw, xs, xw, xcn, xe, xn, xne, rc, rn;
        {
            const UpIn<W> q0 = load(0, j0 - 1), q1 = load(1, j0 - 1), q2 = load(0, j0), q3 = load(1, j0),
                          q4 = load(2, j0), q5 = load(1, j0 + 1), q6 = load(2, j0 + 1);
            xsw = up_eval_t<T, true, PRE, VK>(q0, dl, idl, om, L.z);
            xs = up_eval_t<T, true, PRE, VK>(q1, dl, idl, om, L.z);
            xw = up_eval_t<T, true, PRE, VK>(q2, dl, idl, om, L.z);
            xcn = up_eval_t<T, true, PRE, VK>(q3, dl, idl, om, L.z);
            xe = up_eval_t<T, true, PRE, VK>(q4, dl, idl, om, L.z);
            xn = up_eval_t<T, true, PRE, VK>(q5, dl, idl, om, L.z);
            xne = up_eval_t<T, true, PRE, VK>(q6, dl, idl, om, L.z);
            rc = q3.r;
            rn = q5.r;
        }
        // Coarse window: x_c on the coarse columns kc0 + d (d < 3; two suffice when ai is odd)
        // and the coarse rows R0, R0 + 1 with R0 = (aj + 1) >> 1, which hold every coarse value
        // that the P1 interpolation needs at the step's new points (ai-1, aj+1), (ai, aj+2),
        // (ai+1, aj+2). The window moves by one coarse row every second fine row, so each
        // coarse value is loaded once per column walk instead of at every fine point (in FP32
        // mode too: the loads saved outweigh the registers, 1.50 -> 1.24 ms at 1024^2 x 512). The
        // parities of ai and aj (uniform) are compile-time in the code below.
        const int kc0 = (ai - 1) >> 1;
        const int nc = C.n;
        unsigned occ[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) occ[d] = (((unsigned)(kc0 + d) << lgST) + L.s0) * E;
        // rows outside the grid are clamped onto it: their values are never used (x2_at)
        auto rload = [&](int d, int bj) -> W { return *cboff(row_of(rin, clampi(bj, 0, nF), sf, lgR), ofn[d]); };
        auto mload = [&](int d, int bj) -> double {
            return uload<UNI>(F.mt, (long)clampi(bj, 0, nF) * sf + ai - 1 + d);
        };
        auto kload = [&](int d, int bj) -> double {   // Khat diagonal (VK)
            return uload<UNI>(F.kt, (long)clampi(bj, 0, nF) * sf + ai - 1 + d);
        };
        auto walk = [&](auto aodd_) {
            constexpr bool AODD = decltype(aodd_)::value;
            constexpr int NCOL = AODD ? 2 : 3;
            W cw[3][2];
            auto load_crow = [&](int cr, auto e_) {
                constexpr int e = decltype(e_)::value;
                const int cc = clampi(cr, 0, nc);   // rows past the grid feed only discarded points
#pragma unroll
                for (int d = 0; d < 3; ++d)
                    cw[d][e] = d < NCOL ? *cboff(row_of(xc, cc, sc, lgR), occ[d]) : sv_zero<T>();
            };
            // the window of the step before the first one: the first step moves it up when j0 is odd
            int R0 = j0 >> 1;
            load_crow(R0, std::integral_constant<int, 0>());
            load_crow(R0 + 1, std::integral_constant<int, 1>());
            // P x_c at fine column ai-1+c on a row of parity ROWODD whose coarse row is R0 + e:
            // coarse column offset d and column parity of the fine column follow from AODD
            auto px = [&](auto c_, auto rowodd_, auto e_) -> W {
                constexpr int c = decltype(c_)::value;
                constexpr bool ROWODD = decltype(rowodd_)::value;
                constexpr int e = decltype(e_)::value;
                constexpr int d = c == 0 ? 0 : (c == 2 ? 1 : (AODD ? 0 : 1));
                constexpr bool CODD = AODD ? (c == 1) : (c != 1);
                const W a0 = cw[d][e];
                if (!CODD && !ROWODD) return a0;
                constexpr int d1 = CODD ? d + 1 : d;
                constexpr int e1 = ROWODD ? e + 1 : e;
                return sv_scale((T)0.5, sv_add(a0, cw[d1][e1]));
            };
            auto x2_at = [&](int bj, const W& r, double mc, double kc, const W& pxv, auto mass_) -> W {
                constexpr bool MASS = decltype(mass_)::value;
                if (bj < 0 || bj > nF) return sv_zero<T>();
                if constexpr (!PRE) return pxv;
                const T dlk = VK ? (T)kc : dl, idlk = VK ? (T)1 / dlk : idl;
                return sv_add(jacobi_t<T, MASS>(dlk, idlk, om, mc, L.z, r), pxv);
            };
            // one fine row aj < row1 (inside the chunk: computed and stored; past it: loads only)
            auto step = [&](int aj, auto ajodd_) {
                constexpr bool AJODD = decltype(ajodd_)::value;
                const bool here = aj < sr.row1, more = aj + 1 < sr.row1;
                if (AJODD) {  // R0 = (aj + 1) / 2 moved up by one: shift the coarse window
#pragma unroll
                    for (int d = 0; d < 3; ++d) cw[d][0] = cw[d][1];
                    R0 += 1;
                    load_crow(R0 + 1, std::integral_constant<int, 1>());
                }
                // (PRE = false: only the centre column's r, for the post-smoothing)
                const W r1 = rload(1, aj + 2);
                const W r0 = PRE ? rload(0, aj + 1) : sv_zero<T>(), r2 = PRE ? rload(2, aj + 2) : sv_zero<T>();
                const double m0 = PRE ? mload(0, aj + 1) : 0.0, m1 = PRE ? mload(1, aj + 2) : 0.0,
                             m2 = PRE ? mload(2, aj + 2) : 0.0;
                const double k0 = (PRE && VK) ? kload(0, aj + 1) : 0.0, k1 = (PRE && VK) ? kload(1, aj + 2) : 0.0,
                             k2 = (PRE && VK) ? kload(2, aj + 2) : 0.0;
                issue_fence();
                W out = sv_zero<T>();
                if (here && aj > 0 && aj < nF) {
                    const long node = (long)aj * sf + ai;
                    const MRow m = mrow<UNI>(F, node);
                    MRow kr{};
                    T dlc = dl, idlc = idl;
                    if constexpr (VK) {  // the node's Khat row and diagonal
                        kr = krow<UNI>(F, node);
                        dlc = (T)kr.c;
                        idlc = (T)1 / dlc;
                    }
                    if (m.any())
                        out = post_smooth_t<T, true, VK>(m, nu, dlc, idlc, om, L.z, rc, xcn, xe, xw, xn, xs, xne, xsw,
                                                         kr);
                    else
                        out = post_smooth_t<T, false, VK>(m, nu, dlc, idlc, om, L.z, rc, xcn, xe, xw, xn, xs, xne, xsw,
                                                          kr);
                    if (dotmode != DOT_NONE) sv_dot_acc(acc, out, rc, dotmode == DOT_HERM);
                }
                if (here) nt_store(boff(row_of(xout, aj, sf, lgR), ofn[1]), out);
                if (more) {
                    // aj even: row aj + 1 (column ai-1) is odd on coarse row R0, row aj + 2 even on
                    // R0 + 1; aj odd: aj + 1 even on R0, aj + 2 odd on R0
                    using RW = std::integral_constant<bool, !AJODD>;
                    using RCE = std::integral_constant<bool, AJODD>;
                    using EW = std::integral_constant<int, 0>;
                    using ECE = std::integral_constant<int, AJODD ? 0 : 1>;
                    xsw = xw;
                    xs = xcn;
                    xcn = xn;
                    rc = rn;
                    xe = xne;
                    rn = r1;
                    const W p0 = px(std::integral_constant<int, 0>(), RW(), EW());
                    const W p1 = px(std::integral_constant<int, 1>(), RCE(), ECE());
                    const W p2 = px(std::integral_constant<int, 2>(), RCE(), ECE());
                    if (PRE && (nzbits(m0) | nzbits(m1) | nzbits(m2)) != 0) {  // one branch per row
                        xw = x2_at(aj + 1, r0, m0, k0, p0, std::true_type());
                        xn = x2_at(aj + 2, r1, m1, k1, p1, std::true_type());
                        xne = x2_at(aj + 2, r2, m2, k2, p2, std::true_type());
                    } else {
                        xw = x2_at(aj + 1, r0, m0, k0, p0, std::false_type());
                        xn = x2_at(aj + 2, r1, m1, k1, p1, std::false_type());
                        xne = x2_at(aj + 2, r2, m2, k2, p2, std::false_type());
                    }
                }
            };
            int aj = j0;
            if (aj & 1) {  // j0 < row1 here
                step(aj, std::true_type());
                ++aj;
            }
            // four rows per iteration: the window's values then come back to the registers they
            // started in after fewer register moves than with two (1.04 -> 1.00 ms at 1024^2 x 512)
            for (; aj < sr.row1; aj += 4) {
                step(aj, std::false_type());
                step(aj + 1, std::true_type());
                step(aj + 2, std::false_type());
                step(aj + 3, std::true_type());
            }
        };
        if (ai & 1)
            walk(std::true_type());
        else
            walk(std::false_type());
    } else if (ai < sf) {
        const unsigned oc = (((unsigned)ai << lgST) + L.s0) * E;
        for (int aj = sr.row0; aj < sr.row1; ++aj) *boff(row_of(xout, aj, sf, lgR), oc) = sv_zero<T>();
    }
    if (dotmode != DOT_NONE) store_dot_partials<V>(acc, part, vb, ST, blockIdx.y, SC);
}

// ---------------------------------------------------------------- operator apply

// y = A x and the dot partials of (x, A x) for the two adjacent columns a0 = 2 pc and a0 + 1
// of a team (the grid's columns 0..n in pairs; the last pair has one column): the rolling
// window spans columns a0-1 .. a0+2, so each row loads four new points for two outputs
// instead of three for one. The window is kept in row slots modulo 4 (row aj in slot
// (aj - j0 + 1) & 3) with the row loop unrolled by 4, so it is never moved between registers.
// Boundary columns and rows give 0. VK: Khat from the level's stencil table (per-region Khat).
template <typename T, bool UNI, bool VK>
__global__ void __launch_bounds__(kBlock) k_matvec(SlotArgs sa, LvArgs F, const void* x_, void* y_, int dotmode,
                                                   double* part) {
    using W = SV<T>;
    constexpr int V = W::V;
    const W* x = (const W*)x_;
    W* y = (W*)y_;
    const int ST = sa.ST, lgST = sa.lgST, lgR = lgST - (V - 1), SC = sa.slot_chunk;
    const SlotLane<T> L = slot_lane<T>(sa);
    const int vb = virtual_block(sa.remap);
    const T nu = (T)sa.nu;
    const int sf = F.side, nF = F.n;
    const unsigned E = sizeof(typename Vec2<T>::type);
    double acc[V][3] = {};
    const SweepRange sr = sweep_range(vb, sa.col_groups, sa.per_step, sa.rows_per_chunk, F.side);
    int pc = sr.col0 + L.ln;
    if (UNI) pc = __builtin_amdgcn_readfirstlane(pc);
    const int a0 = 2 * pc;
    if (a0 <= nF && sr.row0 < sr.row1) {
        const bool two = a0 + 1 <= nF;   // the pair's second column exists
        // columns a0-1, a0, a0+1, a0+2, clamped onto the grid (values there never used)
        unsigned oc[4];
#pragma unroll
        for (int d = 0; d < 4; ++d) oc[d] = (((unsigned)clampi(a0 - 1 + d, 0, nF) << lgST) + L.s0) * E;
        // rows outside the grid are clamped onto it (loaded on every path, never used)
        auto ld = [&](int d, int bj) -> W { return *cboff(row_of(x, clampi(bj, 0, nF), sf, lgR), oc[d]); };
        const int j0 = sr.row0;
        W Wc[4], C0[4], C1[4], Ec[4];
        Wc[0] = ld(0, j0 - 1);
        C0[0] = ld(1, j0 - 1);
        C1[0] = ld(2, j0 - 1);
        Wc[1] = ld(0, j0);
        C0[1] = ld(1, j0);
        C1[1] = ld(2, j0);
        Ec[1] = ld(3, j0);
        C0[2] = ld(1, j0 + 1);
        C1[2] = ld(2, j0 + 1);
        Ec[2] = ld(3, j0 + 1);
        const bool in0 = a0 > 0 && a0 < nF, in1 = a0 + 1 < nF;
        auto row = [&](int aj, auto r_) {
            constexpr int r = decltype(r_)::value;  // slot of row aj - 1
            constexpr int s0 = r, s1 = (r + 1) & 3, s2 = (r + 2) & 3, s3 = (r + 3) & 3;
            // next row's new points, loaded before this row is computed (on every path)
            Wc[s2] = ld(0, aj + 1);
            C0[s3] = ld(1, aj + 2);
            C1[s3] = ld(2, aj + 2);
            Ec[s3] = ld(3, aj + 2);
            issue_fence();
            if (aj >= sr.row1) return;
            W out0 = sv_zero<T>(), out1 = sv_zero<T>();
            if (aj > 0 && aj < nF) {
                if (in0) {
                    const long nd0 = (long)aj * sf + a0;
                    out0 = apply_A<T, VK>(mrow<UNI>(F, nd0), nu, L.z, C0[s1], C1[s1], Wc[s1], C0[s2], C0[s0], C1[s2],
                                          Wc[s0], VK ? krow<UNI>(F, nd0) : MRow{});
                    if (dotmode != DOT_NONE) sv_dot_acc(acc, C0[s1], out0, dotmode == DOT_HERM);
                }
                if (in1) {
                    const long nd1 = (long)aj * sf + a0 + 1;
                    out1 = apply_A<T, VK>(mrow<UNI>(F, nd1), nu, L.z, C1[s1], Ec[s1], C0[s1], C1[s2], C1[s0], Ec[s2],
                                          C0[s0], VK ? krow<UNI>(F, nd1) : MRow{});
                    if (dotmode != DOT_NONE) sv_dot_acc(acc, C1[s1], out1, dotmode == DOT_HERM);
                }
            }
            if (y) {
                *boff(row_of(y, aj, sf, lgR), oc[1]) = out0;
                if (two) *boff(row_of(y, aj, sf, lgR), oc[2]) = out1;
            }
        };
        for (int aj = j0; aj < sr.row1; aj += 4) {
            row(aj, std::integral_constant<int, 0>());
            row(aj + 1, std::integral_constant<int, 1>());
            row(aj + 2, std::integral_constant<int, 2>());
            row(aj + 3, std::integral_constant<int, 3>());
        }
    }
    if (dotmode != DOT_NONE) store_dot_partials<V>(acc, part, vb, ST, blockIdx.y, SC);
}

// ---------------------------------------------------------------- per-slot scalars

// Sum the partials of every workgroup in a fixed order and combine them into a generic
// scalar: Hermitian u^H v = (s1 + s2) + i s3, bilinear u^T v = (s1 - s2) + i s3, and for
// slot 0 the two real dot products (s1, s2).
// Stage 1: workgroup (x, y) sums partial rows [y nblk / RB, (y+1) nblk / RB) for SG slots
// (threads: SG slots x 256/SG row lanes, lanes combined in a fixed order) into part2[y][s].
// Workgroups z = 1 do the same for a second set (part_b, nblk_b, RB_b, part2_b); each set
// keeps its own RB (workgroups with y >= RB of their set have nothing to do).
struct Dots1Set {
    const double* part;
    int nblk, RB;
    double* part2;
};
__global__ void __launch_bounds__(kBlock) k_reduce_dots1(Dots1Set a, Dots1Set b, int S) {
    __shared__ double red[3][kBlock];
    const Dots1Set& d = blockIdx.z == 0 ? a : b;
    const double* part = d.part;
    const int nblk = d.nblk, RB = d.RB;
    double* part2 = d.part2;
    if ((int)blockIdx.y >= RB) return;  // (uniform in the workgroup)
    const int SG = S < 64 ? S : 64, RL = kBlock / SG;
    const int sl = threadIdx.x % SG, rl = threadIdx.x / SG;
    const int s = blockIdx.x * SG + sl;
    const int b0 = (int)((long)blockIdx.y * nblk / RB), b1 = (int)((long)(blockIdx.y + 1) * nblk / RB);
    double s1 = 0, s2 = 0, s3 = 0;
    // rows b0 + rl, b0 + rl + RL, ... added in that order; the loads of kReduceBatch rows are
    // issued together (rows past b1 clamped onto the first one, loaded and not added)
    for (int b = b0 + rl; b < b1; b += RL * kReduceBatch) {
        double v[kReduceBatch][3];
#pragma unroll
        for (int u = 0; u < kReduceBatch; ++u) {
            const int bb = b + u * RL < b1 ? b + u * RL : b;
            const double* o = part + ((size_t)bb * S + s) * 3;
            v[u][0] = o[0];
            v[u][1] = o[1];
            v[u][2] = o[2];
        }
#pragma unroll
        for (int u = 0; u < kReduceBatch; ++u) {
            if (b + u * RL < b1) {
                s1 += v[u][0];
                s2 += v[u][1];
                s3 += v[u][2];
            }
        }
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

// Stage 2: the row sums of part2 per slot, combined into a generic scalar (S = total slots,
// Si = slots per instance). kS2Lanes lanes per slot: lane l adds rows l, l + kS2Lanes, ... in
// that order, then the lane sums are added in lane order.
constexpr int kS2Lanes = 16;

__device__ __forceinline__ double2 dots_combine(double s1, double s2, double s3, int s, int Si, int herm) {
    double2 r;
    if ((s & (Si - 1)) == 0) {
        r.x = s1;
        r.y = s2;
    } else {
        r.x = herm ? (s1 + s2) : (s1 - s2);
        r.y = s3;
    }
    return r;
}

// coef = num / den in generic arithmetic (the Galerkin step's ratio p^H r / p^H A p, whose
// denominator has a positive real part for a nonzero p). A zero denominator gives 0: it occurs
// only for p = 0, i.e. a frequency whose right-hand side vanishes.
__device__ __forceinline__ double2 slot_ratio(double2 a, double2 b, int s, int Si) {
    double2 r;
    if ((s & (Si - 1)) == 0) {
        r.x = (b.x != 0.0) ? a.x / b.x : 0.0;
        r.y = (b.y != 0.0) ? a.y / b.y : 0.0;
    } else {
        double d = b.x * b.x + b.y * b.y;
        r.x = d != 0.0 ? (a.x * b.x + a.y * b.y) / d : 0.0;
        r.y = d != 0.0 ? (a.y * b.x - a.x * b.y) / d : 0.0;
    }
    return r;
}

// Stage 2 of one reduction (out = rows of pa), or of two and their ratio in one launch (RATIO:
// outa = rows of pa, outb = rows of pb, coef = outa / outb per slot).
template <bool RATIO>
__global__ void __launch_bounds__(kBlock) k_reduce_dots2(const double* pa, int RBa, const double* pb, int RBb, int S,
                                                         int Si, int herm, double* outa, double* outb, double* coef) {
    __shared__ double red[6][kBlock];
    const int ln = threadIdx.x % kS2Lanes;
    const int s = blockIdx.x * (kBlock / kS2Lanes) + threadIdx.x / kS2Lanes;
    double v[6] = {0, 0, 0, 0, 0, 0};
    if (s < S) {
        for (int b = ln; b < RBa; b += kS2Lanes) {
            const double* o = pa + ((size_t)b * S + s) * 3;
            v[0] += o[0];
            v[1] += o[1];
            v[2] += o[2];
        }
        if (RATIO) {
            for (int b = ln; b < RBb; b += kS2Lanes) {
                const double* o = pb + ((size_t)b * S + s) * 3;
                v[3] += o[0];
                v[4] += o[1];
                v[5] += o[2];
            }
        }
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) red[c][threadIdx.x] = v[c];
    __syncthreads();
    if (ln == 0 && s < S) {
        double t[6] = {0, 0, 0, 0, 0, 0};
        for (int l = 0; l < kS2Lanes; ++l)
#pragma unroll
            for (int c = 0; c < 6; ++c) t[c] += red[c][threadIdx.x + l];
        const double2 a = dots_combine(t[0], t[1], t[2], s, Si, herm);
        ((double2*)outa)[s] = a;
        if (RATIO) {
            const double2 b = dots_combine(t[3], t[4], t[5], s, Si, herm);
            ((double2*)outb)[s] = b;
            ((double2*)coef)[s] = slot_ratio(a, b, s, Si);
        }
    }
}

// ---------------------------------------------------------------- COCG vector updates

// Workgroup (bx, cy) of the COCG vector kernels covers the slots [cy SC, cy SC + SC) with
// SC = min(ST, kBlock), at the nodes bx NL + nl + k Gx NL (NL = kBlock / SC node lanes per
// slot, Gx = gridDim.x), so every thread keeps one slot. The kernel leaves the squares of the
// new r per slot in part[(bx ST + s) 3 + {0, 1, 2}] = (sum r.x^2, sum r.y^2, 0): the
// Hermitian partials of r^H r (slot 0: the two real systems' squares apart), reduced like the
// other dot partials. CV_XR: x += a (x) p, r -= a (x) q. CV_COPY: r = p.
enum CocgVecMode { CV_XR = 0, CV_COPY = 1 };

template <typename T, int MODE>
__global__ void __launch_bounds__(kBlock) k_cocg_vec(int ST, int Si, size_t nodes, const double* coef, void* x_,
                                                     void* r_, const void* p_, const void* q_, double* part) {
    using T2 = typename Vec2<T>::type;
    __shared__ double red[2][kBlock];
    const int SC = ST < kBlock ? ST : kBlock, NL = kBlock / SC;
    const int ls = threadIdx.x % SC, nl = threadIdx.x / SC;
    const int s = blockIdx.y * SC + ls;
    T2* x = (T2*)x_;
    T2* r = (T2*)r_;
    const T2* p = (const T2*)p_;
    const T2* q = (const T2*)q_;
    GS<T> g{};
    if (MODE == CV_XR) g = gs_from<T>(((const double2*)coef)[s], (s & (Si - 1)) == 0);
    double a0 = 0.0, a1 = 0.0;
    for (size_t nd = (size_t)blockIdx.x * NL + nl; nd < nodes; nd += (size_t)gridDim.x * NL) {
        const size_t id = nd * ST + s;
        T2 rn;
        if (MODE == CV_XR) {
            x[id] = add2(x[id], gs_apply(g, p[id]));
            rn = sub2(r[id], gs_apply(g, q[id]));
        } else {
            rn = p[id];
        }
        r[id] = rn;
        a0 += (double)rn.x * (double)rn.x;
        a1 += (double)rn.y * (double)rn.y;
    }
    red[0][threadIdx.x] = a0;
    red[1][threadIdx.x] = a1;
    __syncthreads();
    if (nl == 0) {
        for (int l = 1; l < NL; ++l) {  // node lanes added in lane order
            a0 += red[0][l * SC + ls];
            a1 += red[1][l * SC + ls];
        }
        double* o = part + ((size_t)blockIdx.x * ST + s) * 3;
        o[0] = a0;
        o[1] = a1;
        o[2] = 0.0;
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

// Stage 2 of the COCG reductions: the rows of part2 summed per slot as in k_reduce_dots2
// (kS2Lanes lanes per slot, lane sums added in lane order), then per slot s, with the
// components c = .x, .y of slot 0 (the real systems k = 0 and k = N/2) treated apart and one
// complex value for s >= 1:
//   COCG_NORM0: nr = r^H r, thr = eta2 nr, act = [nr > 0]           (start: r = the right-hand side)
//   COCG_NORM:  act = act and [nr > thr]; *count += active components (the caller zeroes it)
//   COCG_ALPHA: den = p^T A p, alpha = rho / den where active, 0 elsewhere; *flag = 1 if an active
//             component has |den| <= btol Re(p^H A p) (breakdown of the bilinear form)
//   COCG_RHO:   rho = r^T z
//   COCG_BETA:  beta = r^T z / rho where active, 0 elsewhere; rho = r^T z
// v holds (nr, thr, act) for the norm ops and (rho, alpha or beta) otherwise.

struct CocgScal {
    double2* nr;     // r^H r per component
    double2* thr;    // eta^2 ||Rhat||^2 per component
    double2* act;    // 1 = active, 0 = converged (masked)
    double2* rho;    // r^T z
    double2* coef;   // alpha or beta
    int* count;      // active components after COCG_NORM
    int* flag;       // breakdown
    double eta2, btol;
};

__device__ __forceinline__ double2 gen_div(double2 a, double2 b, bool s0) {
    double2 r;
    if (s0) {
        r.x = b.x != 0.0 ? a.x / b.x : 0.0;
        r.y = b.y != 0.0 ? a.y / b.y : 0.0;
    } else {
        const double d = b.x * b.x + b.y * b.y;
        r.x = d != 0.0 ? (a.x * b.x + a.y * b.y) / d : 0.0;
        r.y = d != 0.0 ? (a.y * b.x - a.x * b.y) / d : 0.0;
    }
    return r;
}

template <int OP>
__global__ void __launch_bounds__(kBlock) k_cocg_stage2(const double* pa, int RB, int S, int Si, CocgScal c) {
    __shared__ double red[3][kBlock];
    const int ln = threadIdx.x % kS2Lanes;
    const int s = blockIdx.x * (kBlock / kS2Lanes) + threadIdx.x / kS2Lanes;
    double v[3] = {0, 0, 0};
    if (s < S) {
        for (int b = ln; b < RB; b += kS2Lanes) {
            const double* o = pa + ((size_t)b * S + s) * 3;
            v[0] += o[0];
            v[1] += o[1];
            v[2] += o[2];
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) red[k][threadIdx.x] = v[k];
    __syncthreads();
    if (ln != 0 || s >= S) return;
    double t[3] = {0, 0, 0};
    for (int l = 0; l < kS2Lanes; ++l)
#pragma unroll
        for (int k = 0; k < 3; ++k) t[k] += red[k][threadIdx.x + l];
    const bool s0 = (s & (Si - 1)) == 0;
    if (OP == COCG_NORM0 || OP == COCG_NORM) {
        const double2 nr = s0 ? make_double2(t[0], t[1]) : make_double2(t[0] + t[1], t[0] + t[1]);
        c.nr[s] = nr;
        double2 act;
        if (OP == COCG_NORM0) {
            c.thr[s] = make_double2(c.eta2 * nr.x, c.eta2 * nr.y);
            act = make_double2(nr.x > 0.0 ? 1.0 : 0.0, nr.y > 0.0 ? 1.0 : 0.0);
        } else {
            const double2 th = c.thr[s], a = c.act[s];
            act = make_double2((a.x != 0.0 && nr.x > th.x) ? 1.0 : 0.0, (a.y != 0.0 && nr.y > th.y) ? 1.0 : 0.0);
            const int n = s0 ? (int)act.x + (int)act.y : (int)act.x;
            if (n) atomicAdd(c.count, n);
        }
        if (!s0) act.y = act.x;
        c.act[s] = act;
        return;
    }
    // bilinear combine of the partials (slot 0: the two real dot products)
    const double2 bl = s0 ? make_double2(t[0], t[1]) : make_double2(t[0] - t[1], t[2]);
    const double2 act = c.act[s];
    if (OP == COCG_ALPHA) {
        double2 al = gen_div(c.rho[s], bl, s0);
        if (s0) {
            const bool bx = act.x != 0.0 && fabs(bl.x) <= c.btol * fabs(t[0]);
            const bool by = act.y != 0.0 && fabs(bl.y) <= c.btol * fabs(t[1]);
            if (bx || by) *c.flag = 1;
            al.x = (act.x != 0.0 && !bx) ? al.x : 0.0;
            al.y = (act.y != 0.0 && !by) ? al.y : 0.0;
        } else {
            const bool bk = act.x != 0.0 && sqrt(bl.x * bl.x + bl.y * bl.y) <= c.btol * (t[0] + t[1]);
            if (bk) *c.flag = 1;
            if (act.x == 0.0 || bk) al = make_double2(0.0, 0.0);
        }
        c.coef[s] = al;
    } else if (OP == COCG_RHO) {
        c.rho[s] = bl;
    } else {
        double2 be = gen_div(bl, c.rho[s], s0);
        if (s0) {
            be.x = act.x != 0.0 ? be.x : 0.0;
            be.y = act.y != 0.0 ? be.y : 0.0;
        } else if (act.x == 0.0) {
            be = make_double2(0.0, 0.0);
        }
        c.coef[s] = be;
        c.rho[s] = bl;
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
    L.kt = p.vk ? (const double*)(ws + p.lev[l].off_kt) : nullptr;
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
    // levels l0 .. L-1 (side <= kSmallSide, l0 >= 1) run in one k_vc_small launch
    int l0 = L;
    for (int l = 1; l < L; ++l)
        if (p.lev[l].side <= kSmallSide) {
            l0 = l;
            break;
        }
    if (L - l0 > kMaxSmall) l0 = L;  // (sides 33, 17, 9, 5, 3: never more than kMaxSmall)
    // restriction sweep
    for (int l = 0; l + 1 < L && l < l0; ++l) {
        const void* rin = (l == 0) ? r0 : (const void*)(ws + p.lev[l].off_r);
        void* rout = ws + p.lev[l + 1].off_r;
        Geom g = slot_geom(p.lev[l + 1].side, p.ST, p.fp32 ? 2 : 1, p.target_down);
        SlotArgs sa = mk_slot(p, ws, g);
        dim3 grid(g.blocks, g.chunks);
        int kid = (l == 0) ? KID_DOWN0 : KID_DOWNC;
        tm_begin(p, kid, st);
        LvArgs Fl = host_lv(p, ws, l), Cl = host_lv(p, ws, l + 1);
        bool uni = g.slot_chunk >= 64;
        if (!p.vc_pre) {
            if (p.fp32) {
                if (uni)
                    hipLaunchKernelGGL((k_vc_restrict<float, true>), grid, dim3(kBlock), 0, st, sa, Fl, Cl, rin, rout);
                else
                    hipLaunchKernelGGL((k_vc_restrict<float, false>), grid, dim3(kBlock), 0, st, sa, Fl, Cl, rin, rout);
            } else {
                if (uni)
                    hipLaunchKernelGGL((k_vc_restrict<double, true>), grid, dim3(kBlock), 0, st, sa, Fl, Cl, rin, rout);
                else
                    hipLaunchKernelGGL((k_vc_restrict<double, false>), grid, dim3(kBlock), 0, st, sa, Fl, Cl, rin,
                                       rout);
            }
        } else {
            auto down = [&](auto t_, auto uni_, auto vk_) {
                using T = decltype(t_);
                constexpr bool U = decltype(uni_)::value, VK = decltype(vk_)::value;
                hipLaunchKernelGGL((k_vc_down<T, U, VK>), grid, dim3(kBlock), 0, st, sa, Fl, Cl, rin, rout);
            };
            auto down_u = [&](auto t_, auto uni_) {
                if (p.vk) down(t_, uni_, std::true_type());
                else down(t_, uni_, std::false_type());
            };
            auto down_t = [&](auto t_) {
                if (uni) down_u(t_, std::true_type());
                else down_u(t_, std::false_type());
            };
            if (p.fp32)
                down_t(0.0f);
            else
                down_t(0.0);
        }
        tm_end(p, kid, st);
    }
    if (l0 < L) {
        Geom g = slot_geom(p.lev[l0].side, p.ST, p.fp32 ? 2 : 1, p.target_slot);
        SlotArgs sa = mk_slot(p, ws, g);
        SmallArgs sm;
        sm.count = L - l0;
        sm.pre = p.vc_pre ? 1 : 0;
        int off = 0;
        for (int q = 0; q < sm.count; ++q) {
            const LevelDesc& d = p.lev[l0 + q];
            sm.side[q] = d.side;
            sm.mt[q] = (const double*)(ws + d.off_mt);
            sm.kt[q] = p.vk ? (const double*)(ws + d.off_kt) : nullptr;
            sm.off_r[q] = off;
            sm.off_x[q] = off + (int)d.nodes;
            off += 2 * (int)d.nodes;
        }
        sm.off_t = off;
        off += (int)p.lev[l0].nodes;
        const size_t shm = (size_t)off * p.elem;
        tm_begin(p, KID_COARSEST, st);
        if (p.fp32)
            hipLaunchKernelGGL(k_vc_small<float>, dim3(p.ST), dim3(kBlock), shm, st, sa, sm, ws + p.lev[l0].off_r,
                               ws + p.lev[l0].off_x);
        else
            hipLaunchKernelGGL(k_vc_small<double>, dim3(p.ST), dim3(kBlock), shm, st, sa, sm, ws + p.lev[l0].off_r,
                               ws + p.lev[l0].off_x);
        tm_end(p, KID_COARSEST, st);
    } else {
        Geom g = slot_geom(p.lev[L - 1].side, p.ST, p.fp32 ? 2 : 1, p.target_slot);
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
    for (int l = (l0 < L ? l0 : L - 1) - 1; l >= 0; --l) {
        const void* rin = (l == 0) ? r0 : (const void*)(ws + p.lev[l].off_r);
        void* xout = (l == 0) ? x0 : (void*)(ws + p.lev[l].off_x);
        const void* xc = ws + p.lev[l + 1].off_x;
        Geom g = slot_geom(p.lev[l].side, p.ST, p.fp32 ? 2 : 1, p.target_up);   // level 0: p.g_slot0
        SlotArgs sa = mk_slot(p, ws, g);
        dim3 grid(g.blocks, g.chunks);
        int dm = (l == 0) ? dotmode : DOT_NONE;
        int kid = (l == 0) ? KID_UP0 : KID_UPC;
        tm_begin(p, kid, st);
        LvArgs Fl = host_lv(p, ws, l), Cl = host_lv(p, ws, l + 1);
        const bool uni = g.slot_chunk >= 64;
        auto up = [&](auto t_, auto uni_, auto pre_, auto vk_) {
            using T = decltype(t_);
            constexpr bool U = decltype(uni_)::value, PRE = decltype(pre_)::value, VK = decltype(vk_)::value;
            hipLaunchKernelGGL((k_vc_up<T, U, PRE, VK>), grid, dim3(kBlock), 0, st, sa, Fl, Cl, rin, xc, xout, dm,
                               part);
        };
        auto up_u = [&](auto t_, auto uni_) {
            using TT = std::true_type;
            using FF = std::false_type;
            if (p.vc_pre) {
                if (p.vk) up(t_, uni_, TT(), TT());
                else up(t_, uni_, TT(), FF());
            } else {
                if (p.vk) up(t_, uni_, FF(), TT());
                else up(t_, uni_, FF(), FF());
            }
        };
        auto up_t = [&](auto t_) {
            if (uni) up_u(t_, std::true_type());
            else up_u(t_, std::false_type());
        };
        if (p.fp32)
            up_t(0.0f);
        else
            up_t(0.0);
        tm_end(p, kid, st);
    }
}

void launch_matvec(const Plan& p, char* ws, const void* x, void* y, int dotmode, double* part, hipStream_t st) {
    const Geom& g = p.g_mv;
    SlotArgs sa = mk_slot(p, ws, g);
    dim3 grid(g.blocks, g.chunks);
    LvArgs Fl = host_lv(p, ws, 0);
    const bool uni = g.slot_chunk >= 64;
    auto mv = [&](auto t_, auto uni_, auto vk_) {
        using T = decltype(t_);
        constexpr bool U = decltype(uni_)::value, VK = decltype(vk_)::value;
        hipLaunchKernelGGL((k_matvec<T, U, VK>), grid, dim3(kBlock), 0, st, sa, Fl, x, y, dotmode, part);
    };
    auto mv_u = [&](auto t_, auto uni_) {
        if (p.vk) mv(t_, uni_, std::true_type());
        else mv(t_, uni_, std::false_type());
    };
    auto mv_t = [&](auto t_) {
        if (uni) mv_u(t_, std::true_type());
        else mv_u(t_, std::false_type());
    };
    if (p.fp32)
        mv_t(0.0f);
    else
        mv_t(0.0);
}

static Dots1Set dots1_set(const Plan& p, double* part, int nblk) {
    // stage 1 writes into the tail of the partial buffer (after the nblk workgroups' partials)
    Dots1Set d;
    d.part = part;
    d.nblk = nblk;
    d.RB = nblk < kReduceRows ? nblk : kReduceRows;
    d.part2 = part + (size_t)nblk * p.ST * 3;
    return d;
}

void launch_reduce_dots(const Plan& p, double* part, int nblk, int dotmode, double* out, hipStream_t st) {
    const Dots1Set d = dots1_set(p, part, nblk);
    const int RB = d.RB;
    const int SG = p.ST < 64 ? p.ST : 64;
    const double* part2 = d.part2;
    hipLaunchKernelGGL(k_reduce_dots1, dim3((p.ST + SG - 1) / SG, RB, 1), dim3(kBlock), 0, st, d, d, p.ST);
    const int grid = (p.ST + kBlock / kS2Lanes - 1) / (kBlock / kS2Lanes);
    hipLaunchKernelGGL(k_reduce_dots2<false>, dim3(grid), dim3(kBlock), 0, st, part2, RB, (const double*)nullptr, 0,
                       p.ST, p.S, dotmode == DOT_HERM ? 1 : 0, out, (double*)nullptr, (double*)nullptr);
}

void launch_reduce_ratio(const Plan& p, double* pa, int na, double* pb, int nb, int dotmode, double* num, double* den,
                         double* coef, hipStream_t st) {
    const Dots1Set a = dots1_set(p, pa, na), b = dots1_set(p, pb, nb);
    const int SG = p.ST < 64 ? p.ST : 64;
    hipLaunchKernelGGL(k_reduce_dots1, dim3((p.ST + SG - 1) / SG, a.RB > b.RB ? a.RB : b.RB, 2), dim3(kBlock), 0, st, a, b,
                       p.ST);
    const int grid = (p.ST + kBlock / kS2Lanes - 1) / (kBlock / kS2Lanes);
    hipLaunchKernelGGL(k_reduce_dots2<true>, dim3(grid), dim3(kBlock), 0, st, (const double*)a.part2, a.RB,
                       (const double*)b.part2, b.RB, p.ST, p.S, dotmode == DOT_HERM ? 1 : 0, num, den, coef);
}

// Workgroups along the nodes of the COCG vector kernels (rows of their norm partials).
int cocg_rows(const Plan& p) {
    const int SC = p.ST < kBlock ? p.ST : kBlock, NL = kBlock / SC, CY = p.ST / SC;
    long gx = 8192 / CY;
    const long need = (long)((p.nodes + NL - 1) / NL);
    if (gx > need) gx = need;
    if (gx > kCocgRows) gx = kCocgRows;
    return gx < 1 ? 1 : (int)gx;
}

void launch_cocg_vec(const Plan& p, int mode, const double* coef, void* x, void* r, const void* src, const void* q,
                     double* part, hipStream_t st) {
    const int SC = p.ST < kBlock ? p.ST : kBlock;
    dim3 grid(cocg_rows(p), p.ST / SC);
    if (p.fp32) {
        if (mode == CV_XR)
            hipLaunchKernelGGL((k_cocg_vec<float, CV_XR>), grid, dim3(kBlock), 0, st, p.ST, p.S, p.nodes, coef, x, r,
                               src, q, part);
        else
            hipLaunchKernelGGL((k_cocg_vec<float, CV_COPY>), grid, dim3(kBlock), 0, st, p.ST, p.S, p.nodes, coef, x,
                               r, src, q, part);
    } else {
        if (mode == CV_XR)
            hipLaunchKernelGGL((k_cocg_vec<double, CV_XR>), grid, dim3(kBlock), 0, st, p.ST, p.S, p.nodes, coef, x, r,
                               src, q, part);
        else
            hipLaunchKernelGGL((k_cocg_vec<double, CV_COPY>), grid, dim3(kBlock), 0, st, p.ST, p.S, p.nodes, coef, x,
                               r, src, q, part);
    }
}

void launch_cocg_reduce(const Plan& p, double* part, int nblk, int op, const CocgScalars& cs, hipStream_t st) {
    const Dots1Set d = dots1_set(p, part, nblk);
    const int SG = p.ST < 64 ? p.ST : 64;
    hipLaunchKernelGGL(k_reduce_dots1, dim3((p.ST + SG - 1) / SG, d.RB, 1), dim3(kBlock), 0, st, d, d, p.ST);
    CocgScal c;
    c.nr = (double2*)cs.nr;
    c.thr = (double2*)cs.thr;
    c.act = (double2*)cs.act;
    c.rho = (double2*)cs.rho;
    c.coef = (double2*)cs.coef;
    c.count = cs.count;
    c.flag = cs.flag;
    c.eta2 = cs.eta2;
    c.btol = cs.btol;
    const int grid = (p.ST + kBlock / kS2Lanes - 1) / (kBlock / kS2Lanes);
    const double* p2 = d.part2;
    switch (op) {
        case COCG_NORM0:
            hipLaunchKernelGGL(k_cocg_stage2<COCG_NORM0>, dim3(grid), dim3(kBlock), 0, st, p2, d.RB, p.ST, p.S, c);
            break;
        case COCG_NORM:
            hipLaunchKernelGGL(k_cocg_stage2<COCG_NORM>, dim3(grid), dim3(kBlock), 0, st, p2, d.RB, p.ST, p.S, c);
            break;
        case COCG_ALPHA:
            hipLaunchKernelGGL(k_cocg_stage2<COCG_ALPHA>, dim3(grid), dim3(kBlock), 0, st, p2, d.RB, p.ST, p.S, c);
            break;
        case COCG_RHO:
            hipLaunchKernelGGL(k_cocg_stage2<COCG_RHO>, dim3(grid), dim3(kBlock), 0, st, p2, d.RB, p.ST, p.S, c);
            break;
        default:
            hipLaunchKernelGGL(k_cocg_stage2<COCG_BETA>, dim3(grid), dim3(kBlock), 0, st, p2, d.RB, p.ST, p.S, c);
            break;
    }
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
