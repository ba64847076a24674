// Time-axis kernels.
//
//  k_forward  : fused residual sweep and packed real DFT along time. For every node
//               (a team of threads per node) and every time level it evaluates
//                 R^n = f^n - M (u^n - u^{n-1}) / tau - K(u^n),  u^0 = u^N
//               (Problem 1, eq. (disc1)), with the nonlinear P1 operator of Sec. 4
//                 K(u)_i = sum_{T ni i} |T| nu_T(|grad u_T|^2) grad u_T . grad phi_i,
//               accumulates ||R||^2 and ||F||^2 in FP64, then transforms the node's N
//               residual values to the packed half spectrum (remark rem:parallel) by a
//               half-length complex FFT in LDS.
//  k_inverse  : (1/N) inverse packed DFT of a slot vector, scaled per slot by a generic
//               coefficient, added to (or stored into) the node-major iterate.
//  k_transpose: time-major [N][nodes] <-> node-major [nodes][N].
//  k_apply_K  : K(u) slice by slice on the time-major layout.
//
// Geometry on the uniform grid (h = 1/n, |T| = h^2/2): with G = h grad u_T (node
// differences) and g~ = h grad phi (integer vectors), |T| nu grad u . grad phi = nu G.g~ / 2,
// and |grad u|^2 = n^2 |G|^2.
#include <algorithm>
#include <type_traits>

#include "pt_device.h"

namespace pt {

// ---------------------------------------------------------------- in-LDS complex FFT

// Forward (unnormalised) complex DFT of length S of the team's buffer a in LDS, Stockham
// radix-4 stages and one radix-2 stage when log2 S is odd; b is scratch. tw[k] =
// exp(-2 pi i k / N) for k < N (so exp(-2 pi i m / S) = tw[2 m]). Every thread of the
// workgroup must call it (it synchronises the workgroup). Returns the result buffer.
// Every lane of the team (S/4 lanes) owns exactly one butterfly of each radix-4 stage and
// two of the radix-2 stage: the twiddles of a lane do not change from one node to the
// next, so they are read from the table once per kernel and kept in registers (LaneFft)
// instead of being fetched for every transform.
constexpr int kFftMaxR4 = 5;  // radix-4 stages for S <= 1024

template <typename T2> struct LaneFft {
    T2 w[kFftMaxR4][3];
    T2 w2[2];
};

template <typename T2> __device__ __forceinline__ LaneFft<T2> lane_fft_twiddles(const T2* tw, int S, int lt, int TS) {
    LaneFft<T2> L;
    int Ns = 1;
#pragma unroll
    for (int st = 0; st < kFftMaxR4; ++st) {
        const bool on = Ns * 4 <= S;
        const int k = lt & (Ns - 1), stp = on ? S / (2 * Ns) : 0;
        L.w[st][0] = tw[k * stp];
        L.w[st][1] = tw[2 * k * stp];
        L.w[st][2] = tw[3 * k * stp];
        if (on) Ns *= 4;
    }
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int j = lt + h * TS, k = j & (Ns - 1);
        L.w2[h] = (Ns < S) ? tw[(k * (S / Ns)) & (2 * S - 1)] : tw[0];
    }
    return L;
}

template <typename T2>
__device__ __forceinline__ T2* fft_lane(T2* a, T2* b, int S, int lt, int TS, const LaneFft<T2>& L) {
    int Ns = 1;
    const int Q = S >> 2;
#pragma unroll
    for (int st = 0; st < kFftMaxR4; ++st) {
        if (Ns * 4 > S) break;
        if (lt < Q) {
            const int j = lt, k = j & (Ns - 1);
            T2 v0 = a[j], v1 = a[j + Q], v2 = a[j + 2 * Q], v3 = a[j + 3 * Q];
            if (st > 0) {
                v1 = cmul(v1, L.w[st][0]);
                v2 = cmul(v2, L.w[st][1]);
                v3 = cmul(v3, L.w[st][2]);
            }
            T2 t0 = add2(v0, v2), t1 = sub2(v0, v2), t2 = add2(v1, v3), t3 = mul_mi(sub2(v1, v3));
            const int idx = (j / Ns) * Ns * 4 + k;
            b[idx] = add2(t0, t2);
            b[idx + Ns] = add2(t1, t3);
            b[idx + 2 * Ns] = sub2(t0, t2);
            b[idx + 3 * Ns] = sub2(t1, t3);
        }
        __syncthreads();
        T2* t = a;
        a = b;
        b = t;
        Ns *= 4;
    }
    if (Ns < S) {
        const int H = S >> 1;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int j = lt + h * TS;
            if (j < H) {
                const int k = j & (Ns - 1);
                T2 v0 = a[j];
                T2 v1 = cmul(a[j + H], L.w2[h]);
                const int idx = (j / Ns) * Ns * 2 + k;
                b[idx] = add2(v0, v1);
                b[idx + Ns] = sub2(v0, v1);
            }
        }
        __syncthreads();
        T2* t = a;
        a = b;
        b = t;
    }
    return a;
}

// Ordering point for LDS data exchanged between the lanes of one wavefront: LDS accesses of a
// wavefront are carried out in issue order, so it is enough that the compiler keeps them in
// program order here (no instruction is emitted and no other wavefront is waited for).
__device__ __forceinline__ void wave_lds_sync() {
    asm volatile("" ::: "memory");
    __builtin_amdgcn_wave_barrier();
}

// fft_lane on the S/4 lanes lt of one wavefront (S/4 <= 64 lanes per transform, so a
// transform never spans two wavefronts), with the input of the first radix-4 stage in
// registers, v[c] = z_{lt + c S/4}, and LDS-ordering points instead of workgroup barriers
// between the stages. tw: the first S entries of the twiddle table w^i = exp(-2 pi i / N)
// (read by a final radix-2 stage), followed by the stage runs of the radix-4 stages after the
// first (w^(c k S/(2 Ns)) at [3 Ns-run offset + (c-1) Ns + k], the entries of
// lane_fft_twiddles). lgS = log2 S. a and b hold S values each; the result is in one of them.
template <typename T2>
__device__ __forceinline__ T2* fft_wave_tab(const T2 v[4], T2* a, T2* b, int S, int lgS, int lt, const T2* tw) {
    const int Q = S >> 2;
    // every lane has read its inputs before any lane writes a buffer
    wave_lds_sync();
    {
        T2 t0 = add2(v[0], v[2]), t1 = sub2(v[0], v[2]), t2 = add2(v[1], v[3]), t3 = mul_mi(sub2(v[1], v[3]));
        const int idx = lt * 4;
        a[idx] = add2(t0, t2);
        a[idx + 1] = add2(t1, t3);
        a[idx + 2] = sub2(t0, t2);
        a[idx + 3] = sub2(t1, t3);
    }
    wave_lds_sync();
    int Ns = 4, lgNs = 2;
    const T2* ts = tw + S;  // the stage runs after the first S entries
#pragma unroll
    for (int st = 1; st < kFftMaxR4; ++st) {
        if (Ns * 4 > S) break;
        const int j = lt, k = j & (Ns - 1);
        T2 v0 = a[j], v1 = a[j + Q], v2 = a[j + 2 * Q], v3 = a[j + 3 * Q];
        v1 = cmul(v1, ts[k]);
        v2 = cmul(v2, ts[Ns + k]);
        v3 = cmul(v3, ts[2 * Ns + k]);
        ts += 3 * Ns;
        T2 t0 = add2(v0, v2), t1 = sub2(v0, v2), t2 = add2(v1, v3), t3 = mul_mi(sub2(v1, v3));
        const int idx = (j >> lgNs) * Ns * 4 + k;
        b[idx] = add2(t0, t2);
        b[idx + Ns] = add2(t1, t3);
        b[idx + 2 * Ns] = sub2(t0, t2);
        b[idx + 3 * Ns] = sub2(t1, t3);
        wave_lds_sync();
        T2* t = a;
        a = b;
        b = t;
        Ns *= 4;
        lgNs += 2;
    }
    if (Ns < S) {
        const int H = S >> 1;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int j = lt + h * Q;
            if (j < H) {
                const int k = j & (Ns - 1);
                T2 v0 = a[j];
                T2 v1 = cmul(a[j + H], tw[(k << (lgS - lgNs)) & (2 * S - 1)]);
                const int idx = (j >> lgNs) * Ns * 2 + k;
                b[idx] = add2(v0, v1);
                b[idx + Ns] = sub2(v0, v1);
            }
        }
        wave_lds_sync();
        return b;
    }
    return a;
}

// Packed real DFT split: X_k of the real series whose half-length transform is z (k = 2q+e
// for the lane's slot pair q), with pw the twiddles exp(-2 pi i k / N) of its two slots.
template <typename T, typename T2>
__device__ __forceinline__ void rfft_split(const T2* z, int S, int q, const T2 pw[2], int conj, T2 X[2]) {
#pragma unroll
    for (int e = 0; e < 2; ++e) {
        const int k = 2 * q + e;
        if (k == 0) {
            T2 z0 = z[0];
            X[e] = mk2<T>(z0.x + z0.y, z0.x - z0.y);
        } else {
            T2 zk = z[k], zc = conj2(z[S - k]);
            T2 E = scale2((T)0.5, add2(zk, zc));
            T2 O = scale2((T)0.5, mul_mi(sub2(zk, zc)));
            X[e] = add2(E, cmul(pw[e], O));
            if (conj) X[e] = conj2(X[e]);
        }
    }
}

// Packed real DFT split for a mirror pair of slots: from z_k and z_{S-k} of the half-length
// transform (index mod S) and w = exp(-2 pi i k / N), the values X_k and X_{S-k} of the real
// series' spectrum. With E = z_k + conj z_{S-k} and O = -i (z_k - conj z_{S-k}), X_k = (E + w O)/2;
// since E and O of slot S-k are the conjugates of those of slot k and w^(S-k) = -conj w^k,
// X_{S-k} = conj(E - w O)/2. At k = 0 the two are X_0 and X_{N/2}, both real.
template <typename T, typename T2>
__device__ __forceinline__ void rfft_mirror(T2 zk, T2 zm, T2 w, T2& Xk, T2& Xm) {
    const T2 zc = conj2(zm);
    const T2 E = add2(zk, zc);
    const T2 t = cmul(w, mul_mi(sub2(zk, zc)));
    Xk = scale2((T)0.5, add2(E, t));
    Xm = conj2(scale2((T)0.5, sub2(E, t)));
}

// Two consecutive slot values (one 16-byte access in FP32).
template <typename T2> struct alignas(16) Pair {
    T2 a, b;
};

// ---------------------------------------------------------------- forward kernel

struct FwdArgs {
    int n, side, N, S, lgS, ts, nb, col_groups, rows_per_chunk, remap, mode;
    int B, ST, lgST;       // instances in the batch, slots per node over all instances (2^lgST)
    size_t nodes;
    double inv_tau, n2;
    const double4* regp;   // [B][kMaxRegions] law parameters of each region (law_nu)
    const double* U;       // [nodes][N]
    const double* F;       // [nodes][N] explicit load or null
    const double* bload;   // [nodes]
    const double* wave;    // [N]
    const double* mt;      // [4][nodes]
    const uint8_t* flags;  // [2 n^2]
    const double* theta;   // [2 n^2] or null
    const double* rec;     // [B][nodes][kRecDoubles] residual-sweep records
    const void* tw;        // T2 [N]
    void* out;             // T2 [nodes][S] or null
    double* rout;          // [nodes][N] or null
    double* part;          // [gridDim.x][2]
};

// 1 / x for x >= 1 with one Newton step: the step squares the estimate's relative error, which
// leaves at most 2.2e-15 relative over [1, 1e300] (pt_device_reciprocals evaluates it on the
// device), far below the residual's own rounding.
__device__ __forceinline__ double rcp_ge1_1(double x) {
    const double r = __builtin_amdgcn_rcp(x);
    return __builtin_fma(r, __builtin_fma(-x, r, 1.0), r);
}

// The two FP64 reciprocals that replace divides, evaluated on a caller's array (device check of
// their accuracy): y[2i] = rcp_ge1_1(x[i]) (the law's 1 / (1 + s^2)), y[2i+1] = fast_rcp(x[i])
// (the Jacobi inverse of the V-cycle).
__global__ void __launch_bounds__(kBlock) k_reciprocals(const double* __restrict__ x, double* __restrict__ y, long n) {
    for (long i = blockIdx.x * (long)kBlock + threadIdx.x; i < n; i += (long)gridDim.x * kBlock) {
        const double v = x[i];
        y[2 * i] = rcp_ge1_1(v);
        y[2 * i + 1] = fast_rcp<double>(v);
    }
}

void launch_reciprocals(const double* x, double* y, long n, hipStream_t st) {
    const long g = std::min<long>((n + kBlock - 1) / kBlock, 65536);
    hipLaunchKernelGGL(k_reciprocals, dim3((unsigned)g), dim3(kBlock), 0, st, x, y, n);
}

// Per-lane state of the column walk for one time value: u on the rows j-1 (s, sw), j
// (w, c, e) and j+1 (nw, n, ne), and the contribution of the three triangles of the cells
// of row j-1 to K at node (i, j).
struct Win {
    double sw, s, w, c, e, nw, n, ne, carry;
};

// ---------------------------------------------------------------- residual-sweep records

// Everything the residual sweep needs at node (i, j) besides u, in one record read through the
// scalar unit: the seven mass-stencil coefficients (centre, E, W, N, S, NE, SW), the load
// amplitude b, and for the triangles T_a(i,j), T_b(i,j), T_a(i-1,j), T_b(i-1,j) the parameters
// of the reluctivity law of the triangle's region, times its theta:
//  - rational law nu = theta (a + b s^2/(1+s^2)) = A - B / (1 + s^2): (A, B) = theta (a + b, b)
//    (rectangle problems: a = nu_a, b = nu_b in nu_rect, a = nu_out, b = 0 elsewhere);
//  - exp-capped law nu = theta (a min(exp(b s^2), c) + d) = A exp(b min(s^2, z)) + D, z = ln(c)/b:
//    (A, b, z, D) = (theta a, b, z, theta d), and (0, 0, inf, theta (a + d)) where the law is
//    constant (a = 0 or b = 0).
// In both, the law is nonlinear exactly where the second (rational) / first (exp-capped) entry
// is nonzero.
template <int LAW> struct NodeRecT {
    static constexpr int P = LAW == PT_NU_EXPCAP ? 4 : 2;   // law parameters per triangle
    double m[7];
    double bl;
    double law[4][P];
};
template <int LAW> constexpr int rec_doubles() { return 8 + 4 * NodeRecT<LAW>::P; }
static_assert(sizeof(NodeRecT<PT_NU_RATIONAL>) == kRecDoubles * sizeof(double), "record size");
static_assert(sizeof(NodeRecT<PT_NU_EXPCAP>) == kRecDoublesExp * sizeof(double), "record size");
using NodeRec = NodeRecT<PT_NU_RATIONAL>;

// Record idx of a table (through the scalar unit when UNI: adjacent words, merged into wide
// scalar loads).
template <bool UNI, int LAW>
__device__ __forceinline__ NodeRecT<LAW> load_rec(const NodeRecT<LAW>* base, size_t idx) {
    const double* p = reinterpret_cast<const double*>(base + idx);
    NodeRecT<LAW> r;
    double* o = &r.m[0];
#pragma unroll
    for (int k = 0; k < rec_doubles<LAW>(); ++k) o[k] = uload<UNI>(p, (size_t)k);
    return r;
}

struct RecArgs {
    int n, side, B;
    size_t nodes;
    const double* mt;      // [4][nodes] fine mass stencil (shared by the instances)
    const double* bload;   // [B][nodes]
    const uint8_t* flags;  // [B][2 n^2]
    const double* theta;   // [2 n^2] or null (one instance)
    const double4* regp;   // [B][kMaxRegions] law parameters of each region (law_nu)
    void* rec;             // [B][nodes] NodeRecT<LAW>
};

template <int LAW>
__global__ void __launch_bounds__(kBlock) k_row_records(RecArgs a) {
    const size_t total = (size_t)a.B * a.nodes, nt = 2 * (size_t)a.n * a.n;
    NodeRecT<LAW>* rec = (NodeRecT<LAW>*)a.rec;
    for (size_t id = blockIdx.x * (size_t)kBlock + threadIdx.x; id < total; id += (size_t)gridDim.x * kBlock) {
        const int b = (int)(id / a.nodes);
        const size_t node = id - (size_t)b * a.nodes;
        const int i = (int)(node % a.side), j = (int)(node / a.side);
        NodeRecT<LAW> r;
        const bool interior = i > 0 && j > 0 && i < a.n && j < a.n;
        const size_t nd = a.nodes, sd = a.side;
        if (interior) {
            r.m[0] = a.mt[node];
            r.m[1] = a.mt[nd + node];
            r.m[2] = a.mt[nd + node - 1];
            r.m[3] = a.mt[2 * nd + node];
            r.m[4] = a.mt[2 * nd + node - sd];
            r.m[5] = a.mt[3 * nd + node];
            r.m[6] = a.mt[3 * nd + node - sd - 1];
        } else {
            for (int k = 0; k < 7; ++k) r.m[k] = 0.0;
        }
        r.bl = a.bload[id];
        for (int t = 0; t < 4; ++t) {
            const int ci = i - (t >> 1), typ = t & 1;   // cells (i, j), (i, j), (i-1, j), (i-1, j)
            double th = 0.0;
            double4 q = make_double4(0.0, 0.0, 0.0, 0.0);
            if (ci >= 0 && ci < a.n && j < a.n) {
                const size_t tri = 2 * ((size_t)j * a.n + ci) + typ;
                th = a.theta ? a.theta[tri] : 1.0;
                q = a.regp[(size_t)b * kMaxRegions + a.flags[(size_t)b * nt + tri]];
            }
            if constexpr (LAW == PT_NU_RATIONAL) {
                r.law[t][0] = th * (q.x + q.y);   // nu = q.x + q.y s^2/(1+s^2) = A - B / (1 + s^2)
                r.law[t][1] = th * q.y;
            } else {
                const bool nl = q.x != 0.0 && q.y != 0.0;
                r.law[t][0] = nl ? th * q.x : 0.0;
                r.law[t][1] = nl ? q.y : 0.0;
                r.law[t][2] = nl ? q.z : 1e300;
                r.law[t][3] = nl ? th * q.w : th * (q.x + q.w);
            }
        }
        rec[id] = r;
    }
}

void launch_row_records(const Plan& p, char* ws, hipStream_t st) {
    RecArgs a;
    a.n = p.n;
    a.side = p.side;
    a.B = p.B;
    a.nodes = p.nodes;
    a.mt = (const double*)(ws + p.lev[0].off_mt);
    a.bload = (const double*)(ws + p.off_b);
    a.flags = (const uint8_t*)(ws + p.off_flags);
    a.theta = p.prob.d_theta;
    a.regp = (const double4*)(ws + p.off_regp);
    a.rec = ws + p.off_rec;
    size_t g = ((size_t)p.B * p.nodes + kBlock - 1) / kBlock;
    if (g > 65536) g = 65536;
    if (p.law == PT_NU_EXPCAP)
        hipLaunchKernelGGL(k_row_records<PT_NU_EXPCAP>, dim3((unsigned)g), dim3(kBlock), 0, st, a);
    else
        hipLaunchKernelGGL(k_row_records<PT_NU_RATIONAL>, dim3((unsigned)g), dim3(kBlock), 0, st, a);
}

// Reluctivity of a triangle from its record entries, s^2 = n^2 |G|^2. NL: the law is evaluated
// without a branch (rational: exactly A where B = 0, since 1 / (1 + s^2) is finite; exp-capped:
// exactly D where A = 0), so that the laws of all triangles of a row form independent chains;
// otherwise every triangle of the row has a constant law (A, resp. D).
template <bool NL, int LAW = PT_NU_RATIONAL>
__device__ __forceinline__ double nu_law(double gx, double gy, double n2, const double* law) {
    if constexpr (LAW == PT_NU_RATIONAL) {
        if constexpr (!NL) return law[0];
        return law[0] - law[1] * rcp_ge1_1(1.0 + n2 * (gx * gx + gy * gy));
    } else {
        if constexpr (!NL) return law[3];
        return law[0] * exp(law[1] * fmin(n2 * (gx * gx + gy * gy), law[2])) + law[3];
    }
}

// lower_three / upper_four with the reluctivity laws of a record: the record of node
// (i, j-1) holds T_b(i,j-1), T_a(i-1,j-1), T_b(i-1,j-1) as its laws 1, 2, 3; the record of
// node (i, j) holds T_a(i,j), T_b(i,j), T_a(i-1,j), T_b(i-1,j) as laws 0..3.
template <int LAW>
__device__ __forceinline__ double lower_three_rec(const Win& v, double n2, const NodeRecT<LAW>& rs) {
    double g4x = v.e - v.c, g4y = v.c - v.s;
    double g5x = v.s - v.sw, g5y = v.c - v.s;
    double g6x = v.c - v.w, g6y = v.w - v.sw;
    return 0.5 * (nu_law<true, LAW>(g4x, g4y, n2, rs.law[1]) * (g4y - g4x) +
                  nu_law<true, LAW>(g5x, g5y, n2, rs.law[2]) * g5y + nu_law<true, LAW>(g6x, g6y, n2, rs.law[3]) * g6x);
}

// whether any of the four laws of a record is nonlinear (uniform per row in a column walk)
template <int LAW>
__device__ __forceinline__ bool rec_nonlinear(const NodeRecT<LAW>& r) {
    constexpr int q = LAW == PT_NU_RATIONAL ? 1 : 0;
    return (nzbits(r.law[0][q]) | nzbits(r.law[1][q]) | nzbits(r.law[2][q]) | nzbits(r.law[3][q])) != 0;
}

template <bool NL, int LAW>
__device__ __forceinline__ double upper_four_rec(const Win& v, double n2, const NodeRecT<LAW>& rc, double& carry_up) {
    double g1x = v.e - v.c, g1y = v.ne - v.e;    // T_a(i,j)
    double g2x = v.ne - v.n, g2y = v.n - v.c;    // T_b(i,j)
    double g3x = v.c - v.w, g3y = v.n - v.c;     // T_a(i-1,j)
    double g4x = v.n - v.nw, g4y = v.nw - v.w;   // T_b(i-1,j)
    double nu1 = nu_law<NL, LAW>(g1x, g1y, n2, rc.law[0]);
    double nu2 = nu_law<NL, LAW>(g2x, g2y, n2, rc.law[1]);
    double nu3 = nu_law<NL, LAW>(g3x, g3y, n2, rc.law[2]);
    double nu4 = nu_law<NL, LAW>(g4x, g4y, n2, rc.law[3]);
    carry_up = 0.5 * (nu2 * (g2y - g2x) + nu3 * g3y + nu4 * g4x);
    return 0.5 * (nu1 * (-g1x) + nu2 * (-g2y) + nu3 * (g3x - g3y)) + v.carry;
}

// Residual sweep: team of TS = S / KP threads per grid column (KP = 1 or 2 time pairs per
// lane); lane lt owns the time pairs (2m, 2m+1), m = lt + TS k. The team walks down its
// column keeping u on rows j-1..j+1 in registers (three new neighbour series per row) and
// carrying the lower triangles' part of K. Rows are processed in batches of kRowBatch so
// that one LDS exchange per batch forms M u^{n-1} from the neighbouring lane's M u^n.
// Writes R in the solver precision (node-major, [node][N]) for the DFT, and/or in double
// (rout), plus the FP64 norm partials. UNI: one column per wavefront. RK: the source is the
// separable b w(t) (RK_WAVE) or an explicit series F (RK_LOAD), or the sweep copies the field
// itself (RK_SIGNAL: no operator, no mass term).
// Every row issues the same vector loads on every path (indexes clamped to the grid where a
// row or column lies outside it; such values are never used), so that the wait for the data
// of a row never also waits for the loads of the rows after it.
// FUSE (KP = 1, 4 <= S <= 256): instead of the time series R, the sweep writes its packed
// real DFT (the output of k_rfft, remark rem:parallel) to a.out: after a row batch the
// workgroup holds the residual of nb x RB nodes in LDS, and S/4 lanes transform each of them
// (nb RB S/4 = 256 lanes), so the series never goes through HBM (a.rout is not written).
constexpr int kRowBatch = 4;
enum ResKind { RK_WAVE = 0, RK_LOAD = 1, RK_SIGNAL = 2 };

template <typename T, bool UNI, int KP, int RK, bool FUSE, int LAW = PT_NU_RATIONAL>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(FUSE && UNI ? 4 : 1)))
k_residual(FwdArgs a, void* rt_) {
    constexpr bool SIG = RK == RK_SIGNAL;
    static_assert(!FUSE || (KP == 1 && !SIG), "the fused transform takes one pair per lane");
    using T2 = typename Vec2<T>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    constexpr int RB = kRowBatch;
    const int TS = a.ts, S = a.S;
    const int lt = threadIdx.x % TS, team = threadIdx.x / TS;
    // per team and row q of a batch, contiguous: rs [S] double2 (residual without the mass
    // term), me / xo [S] double (even / odd time mass products); 32 S bytes
    auto RSp = [&](int c, int q) { return (double2*)(smem_raw + ((size_t)c * RB + q) * 32 * S); };
    auto MEp = [&](int c, int q) { return (double*)(RSp(c, q) + S); };
    auto XOp = [&](int c, int q) { return MEp(c, q) + S; };
    T2* rt = (T2*)rt_;
    // FUSE: the twiddle table (N values) in LDS after the row blocks, read by every stage
    T2* twl = (T2*)(smem_raw + (size_t)a.nb * RB * 32 * S);
    if constexpr (FUSE) {
        // entries 0..S-1 (the split and a final radix-2 stage read only these), then for each
        // radix-4 stage after the first (Ns = 4, 16, ...) its three twiddles w^(c k S/(2 Ns)),
        // c = 1, 2, 3, k < Ns, as three runs of Ns: the lanes of a stage read consecutive
        // entries (at most S further entries, so the N-entry space suffices)
        const T2* tg = (const T2*)a.tw;
        for (int k = threadIdx.x; k < S; k += kBlock) twl[k] = tg[k];
        int o = S;
        for (int Ns = 4, lgNs = 2; Ns * 4 <= S; Ns *= 4, lgNs += 2) {
            const int lgstp = a.lgS - 1 - lgNs;
            for (int e = threadIdx.x; e < 3 * Ns; e += kBlock) {
                const int c = e / Ns + 1, k = e - (c - 1) * Ns;
                twl[o + e] = tg[(c * k) << lgstp];
            }
            o += 3 * Ns;
        }
        // (the first use follows the barrier after the first row batch)
    }
    const double2* U2 = (const double2*)a.U;
    const int vb = virtual_block(a.remap);
    const int side = a.side, n = a.n;
    const long S_ = S;
    double rr = 0.0, ff = 0.0;
    const SweepRange sr = sweep_range(vb, a.col_groups, a.nb, a.rows_per_chunk, side);
    // virtual column vcol = b (n+1) + i: grid column i of batch instance b
    int vcol = sr.col0 + team;
    if (UNI) vcol = __builtin_amdgcn_readfirstlane(vcol);
    const int bi = vcol / side;
    const int i = vcol - bi * side;
    const bool colvalid = vcol < side * a.B, colint = colvalid && i > 0 && i < n;
    // this instance's source waveform (its materials and load are in the records)
    const double* wave = a.wave + (colvalid ? (size_t)bi * a.N : 0);
    // uniform row base + per-lane byte offset of (column i-1+d, instance bi, pair lt + TS k)
    const int lgST = a.lgST;  // 2^lgST time pairs per node over all instances (= slots per node)
    const long STp = a.ST;
    const int bl_ = bi < a.B ? bi : a.B - 1;   // clamped instance and columns for the loads
    unsigned ofs[3][KP];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const int c = i - 1 + d < 0 ? 0 : (i - 1 + d > n ? n : i - 1 + d);
#pragma unroll
        for (int k = 0; k < KP; ++k)
            ofs[d][k] = ((((unsigned)c) << lgST) + (unsigned)(bl_ * S + lt + TS * k)) * (unsigned)sizeof(double2);
    }
    auto rowU = [&](int cj) { return U2 + ((size_t)(cj * side) << lgST); };
    // u of row cj (0 <= cj <= n) on column i-1+d
    auto ldd = [&](int d, int cj, int k) -> double2 {
        return *reinterpret_cast<const double2*>(reinterpret_cast<const char*>(rowU(cj)) + ofs[d][k]);
    };
    // Window of u (both time levels of the lane's pair) on the columns i-1 (Wv), i (Cv) and
    // i+1 (Ev) in row slots modulo 4: row j lives in slot (j - jin + 1) & 3. The row loop
    // below is unrolled by 4, so the slots are compile-time constants and the window is
    // never moved between registers.
    const int jin = sr.row0 > 1 ? sr.row0 : 1;
    double2 Wv[KP][4], Cv[KP][4], Ev[KP][4];
    double carry[KP][2];
    auto win = [&](int k, int h, int s0, int s1, int s2, double cy) -> Win {
        auto g = [h](const double2& x) { return h ? x.y : x.x; };
        return Win{g(Wv[k][s0]), g(Cv[k][s0]), g(Wv[k][s1]), g(Cv[k][s1]), g(Ev[k][s1]),
                   g(Wv[k][s2]), g(Cv[k][s2]), g(Ev[k][s2]), cy};
    };
    using Rec = NodeRecT<LAW>;
    const Rec* recb = (const Rec*)a.rec + (colvalid ? (size_t)bi * a.nodes : 0);
    if (!SIG && colint && jin < sr.row1 && jin < n) {
        const Rec rs = load_rec<UNI, LAW>(recb, (size_t)(jin - 1) * side + i);
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            Wv[k][0] = ldd(0, jin - 1, k);
            Cv[k][0] = ldd(1, jin - 1, k);
            Wv[k][1] = ldd(0, jin, k);
            Cv[k][1] = ldd(1, jin, k);
            Ev[k][1] = ldd(2, jin, k);
            Wv[k][2] = ldd(0, jin + 1, k);
            Cv[k][2] = ldd(1, jin + 1, k);
            Ev[k][2] = ldd(2, jin + 1, k);
#pragma unroll
            for (int h = 0; h < 2; ++h) carry[k][h] = lower_three_rec(win(k, h, 0, 1, 2, 0.0), a.n2, rs);
        }
    }
    // a first row 0 of the chunk is boundary: zero output
    if (sr.row0 == 0 && colvalid) {
#pragma unroll
        for (int k = 0; k < KP; ++k) {
            const int m = lt + TS * k;
            if (a.rout) ((double2*)a.rout)[(long)i * STp + bi * S + m] = make_double2(0.0, 0.0);
            if (rt) rt[(long)i * STp + bi * S + m] = mk2<T>((T)0, (T)0);
            if constexpr (FUSE) ((T2*)a.out)[(long)i * STp + bi * S + m] = mk2<T>((T)0, (T)0);  // its spectrum
        }
    }
    // the source waveform at the lane's time pairs is the same on every row
    double2 wv[KP];
#pragma unroll
    for (int k = 0; k < KP; ++k) wv[k] = ((const double2*)wave)[lt + TS * k];
    for (int jb = jin; jb < sr.row1; jb += RB) {
        unsigned mass_bits = 0;
        auto row = [&](auto q_) {
            constexpr int q = decltype(q_)::value;  // also the slot of row j - 1
            constexpr int s0 = q, s1 = (q + 1) & 3, s2 = (q + 2) & 3, s3 = (q + 3) & 3;
            const int j = jb + q;
            const bool interior = colint && j < sr.row1 && j > 0 && j < n;
            const int node = colvalid ? j * side + i : 0;
            double2 r[KP];
            double mue[KP], muo[KP];
#pragma unroll
            for (int k = 0; k < KP; ++k) {
                r[k] = make_double2(0.0, 0.0);
                mue[k] = muo[k] = 0.0;
            }
            if constexpr (SIG) {
                // the field itself (loaded on every path, row clamped to the grid)
                const int jl = j < n ? j : n;
                double2 uv[KP];
#pragma unroll
                for (int k = 0; k < KP; ++k) uv[k] = ldd(1, jl, k);
                if (interior) {
#pragma unroll
                    for (int k = 0; k < KP; ++k) r[k] = uv[k];
                }
            } else {
                double2 fx[KP];
                if constexpr (RK == RK_LOAD) {
                    // the explicit source series first: waiting for it leaves the neighbour
                    // series of row j+2 in flight
                    const long nl = (long)(j < n ? j : n) * side + i;
                    const double2* F2 = (const double2*)a.F;
#pragma unroll
                    for (int k = 0; k < KP; ++k) fx[k] = F2[nl * S_ + lt + TS * k];
                }
                // the three new neighbour series of row j+2 (clamped to row n at the end of the
                // grid), loaded before this row is computed
                const bool adv = j + 1 < sr.row1 && j + 1 < n;
                const int jn = j + 2 < n ? j + 2 : n;
#pragma unroll
                for (int k = 0; k < KP; ++k) {
                    Wv[k][s3] = ldd(0, jn, k);
                    Cv[k][s3] = ldd(1, jn, k);
                    Ev[k][s3] = ldd(2, jn, k);
                }
                if (interior) {
                    // mass row, load and reluctivity laws of the row: one record
                    const Rec rc = load_rec<UNI, LAW>(recb, (size_t)node);
                    issue_fence();   // both halves of the record requested before either is used
                    const double mc = rc.m[0], mE = rc.m[1], mW = rc.m[2], mN = rc.m[3], mS = rc.m[4],
                                 mNE = rc.m[5], mSW = rc.m[6];
                    const double bl = rc.bl;
                    const bool nl = rec_nonlinear(rc);
                    const bool mass = (nzbits(mc) | nzbits(mE) | nzbits(mW) | nzbits(mN) | nzbits(mS) |
                                       nzbits(mNE) | nzbits(mSW)) != 0;
                    if (mass) mass_bits |= 1u << q;
#pragma unroll
                    for (int k = 0; k < KP; ++k) {
                        const Win p0 = win(k, 0, s0, s1, s2, carry[k][0]), p1 = win(k, 1, s0, s1, s2, carry[k][1]);
                        // mass products first: the whole record is then needed at the top of the row
                        if (mass) {
                            mue[k] = mc * p0.c + mE * p0.e + mW * p0.w + mN * p0.n + mS * p0.s + mNE * p0.ne +
                                     mSW * p0.sw;
                            muo[k] = mc * p1.c + mE * p1.e + mW * p1.w + mN * p1.n + mS * p1.s + mNE * p1.ne +
                                     mSW * p1.sw;
                        }
                        double2 f;
                        if constexpr (RK == RK_LOAD) f = fx[k];
                        else f = make_double2(bl * wv[k].x, bl * wv[k].y);
                        ff += f.x * f.x + f.y * f.y;
                        double cu0, cu1, K0, K1;
                        if (nl) {
                            K0 = upper_four_rec<true>(p0, a.n2, rc, cu0);
                            K1 = upper_four_rec<true>(p1, a.n2, rc, cu1);
                        } else {
                            K0 = upper_four_rec<false>(p0, a.n2, rc, cu0);
                            K1 = upper_four_rec<false>(p1, a.n2, rc, cu1);
                        }
                        r[k] = make_double2(f.x - K0, f.y - K1);
                        if (adv) {
                            carry[k][0] = cu0;
                            carry[k][1] = cu1;
                        }
                    }
                }
            }
#pragma unroll
            for (int k = 0; k < KP; ++k) {
                const int m = lt + TS * k;
                RSp(team, q)[m] = r[k];
                if ((mass_bits >> q) & 1u) {  // (read only for rows with a mass term)
                    MEp(team, q)[m] = mue[k];
                    XOp(team, q)[m] = muo[k];
                }
            }
        };
        static_assert(kRowBatch == 4, "the row window is kept in slots modulo 4");
        row(std::integral_constant<int, 0>());
        row(std::integral_constant<int, 1>());
        row(std::integral_constant<int, 2>());
        row(std::integral_constant<int, 3>());
        __syncthreads();
        if constexpr (!FUSE) {
            // M (u^n - u^{n-1}) = M u^n - M u^{n-1}: the odd-time product of pair m-1 (cyclic)
#pragma unroll 1
            for (int q = 0; q < RB; ++q) {
                const int j = jb + q;
                if (!colvalid || j >= sr.row1) continue;
                const int node = j * side + i;
                const bool interior = colint && j > 0 && j < n;
                const bool mass = (mass_bits >> q) & 1u;
#pragma unroll
                for (int k = 0; k < KP; ++k) {
                    const int m = lt + TS * k;
                    double2 rv = RSp(team, q)[m];
                    if (mass) {
                        const double* xo = XOp(team, q);
                        double mue = MEp(team, q)[m], muo = xo[m];
                        double prev = xo[m == 0 ? S - 1 : m - 1];
                        rv.x -= (mue - prev) * a.inv_tau;
                        rv.y -= (muo - mue) * a.inv_tau;
                    }
                    if (interior) rr += rv.x * rv.x + rv.y * rv.y;
                    if (a.rout) ((double2*)a.rout)[(long)node * STp + bi * S + m] = rv;
                    if (rt) rt[(long)node * STp + bi * S + m] = mk2<T>((T)rv.x, (T)rv.y);
                }
            }
            __syncthreads();
        } else {
            // Node (team, row fq) of the batch on the S/4 lanes fl of one wavefront (S/4 <= 64
            // divides the wavefront): each lane forms the residual, mass difference included,
            // at the four time pairs m = fl + c S/4 that the first radix-4 stage takes from it,
            // so the series goes straight from the row buffers into the butterflies. The node's
            // buffers are touched by its wavefront only, which needs no workgroup barrier
            // between the stages. With TS = S the RB S/4 lanes of a team's RB nodes are the
            // team's own lanes (lane tid: node (tid / S, (tid / (S/4)) % RB)), so the column,
            // instance and mass bits of the node are those of the team. (The lane index is made
            // opaque so that the transform's addresses and twiddles are formed per batch
            // instead of being kept live across the row walk.)
            int tid = threadIdx.x;
            asm volatile("" : "+v"(tid));
            const int F4 = S >> 2;
            const int fq = (tid >> (a.lgS - 2)) & (RB - 1), fl = tid & (F4 - 1);
            const int fj = jb + fq;
            const bool fvalid = colvalid && fj < sr.row1;
            const bool fint = fvalid && colint && fj > 0 && fj < n;
            const bool fmass = (mass_bits >> fq) & 1u;
            const double2* rs = RSp(team, fq);
            const double* me = MEp(team, fq);
            const double* xo = XOp(team, fq);
            T2 z[4];
#pragma unroll
            for (int c = 0; c < 4; ++c) {
                const int m = fl + c * F4;
                double2 rv = rs[m];
                if (fmass) {
                    const double mue = me[m], muo = xo[m], prev = xo[(m - 1) & (S - 1)];
                    rv.x -= (mue - prev) * a.inv_tau;
                    rv.y -= (muo - mue) * a.inv_tau;
                }
                if (fint) rr += rv.x * rv.x + rv.y * rv.y;
                z[c] = mk2<T>((T)rv.x, (T)rv.y);
            }
            const T2* tw = twl;
            const T2* res = fft_wave_tab<T2>(z, (T2*)RSp(team, fq), (T2*)MEp(team, fq), S, a.lgS, fl, tw);
            if (fvalid) {
                // slots k = fl and fl + S/4 (k < S/2) with their mirrors S - k; the lane with
                // k = 0 stores the packed slot 0 (X_0, X_{N/2}) and slot S/2, its own mirror,
                // X_{N/4} = conj z_{S/2}
                T2* outp = (T2*)a.out + ((size_t)fj * side + i) * a.ST + (size_t)bi * S;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int k = fl + h * F4;
                    T2 Xk, Xm;
                    rfft_mirror<T>(res[k], res[(S - k) & (S - 1)], tw[k], Xk, Xm);
                    int km = S - k;
                    if (h == 0 && k == 0) {
                        Xk = mk2<T>(Xk.x, Xm.x);
                        Xm = conj2(res[S >> 1]);
                        km = S >> 1;
                    }
                    outp[k] = Xk;
                    outp[km] = Xm;
                }
            }
            __syncthreads();
        }
    }
    // per-team reduction of the norm partials (fixed order): part[(vb nb + team) 2 + {0, 1}]
    // with vb the virtual workgroup index (column group vb % col_groups); in the row buffers,
    // which are free after the last batch's barrier (the launch gives at least 2 kBlock doubles)
    double (*red)[kBlock] = (double (*)[kBlock])smem_raw;
    red[0][threadIdx.x] = rr;
    red[1][threadIdx.x] = ff;
    __syncthreads();
    for (int w = TS / 2; w > 0; w >>= 1) {
        if (lt < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (lt == 0 && a.part) {
        const size_t o = ((size_t)vb * a.nb + team) * 2;
        a.part[o] = red[0][threadIdx.x];
        a.part[o + 1] = red[1][threadIdx.x];
    }
}

// Packed real DFT along time of node-major real series rt ([node][N], solver precision):
// the half-length complex FFT of z_m = x_{2m} + i x_{2m+1} and the split into X_k
// (remark rem:parallel). Team of S/4 threads per node.
struct RfftArgs {
    int n, side, N, S, ts, nb, col_groups, rows_per_chunk, remap, B, ST, conj;
    const void* rt;   // T2 [nodes][S]
    const void* tw;   // T2 [N]
    void* out;        // T2 [nodes][S]
};

template <typename T>
__global__ void __launch_bounds__(kBlock) k_rfft(RfftArgs a) {
    using T2 = typename Vec2<T>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T2* smem = (T2*)smem_raw;
    const int TS = a.ts, S = a.S, H = S / 2;
    const int lt = threadIdx.x % TS, team = threadIdx.x / TS;
    T2* buf0 = smem + (size_t)team * 2 * S;
    T2* buf1 = buf0 + S;
    const T2* tw = (const T2*)a.tw;
    const Pair<T2>* rtp = (const Pair<T2>*)a.rt;
    Pair<T2>* outp = (Pair<T2>*)a.out;
    const LaneFft<T2> LF = lane_fft_twiddles<T2>(tw, S, lt, TS);
    // the lane owns the slot pairs q = lt + h TS (h = 0, 1): slots 2q, 2q + 1
    T2 pw[2][2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int q = (lt + h * TS) < H ? lt + h * TS : 0;
        pw[h][0] = tw[2 * q];
        pw[h][1] = tw[2 * q + 1];
    }
    const int vb = virtual_block(a.remap);
    const SweepRange sr = sweep_range(vb, a.col_groups, a.nb, a.rows_per_chunk, a.side);
    const int vcol = sr.col0 + team;  // b (n+1) + i
    const bool colvalid = vcol < a.side * a.B;
    const int bi = vcol / a.side, i = vcol - bi * a.side;
    for (int j = sr.row0; j < sr.row1; ++j) {
        const size_t chunk = colvalid ? ((size_t)j * a.side + i) * a.ST + (size_t)bi * S : 0;  // even
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int q = lt + h * TS;
            if (q < H) {
                Pair<T2> v;
                if (colvalid) {
                    v = rtp[chunk / 2 + q];
                } else {
                    v.a = mk2<T>(0, 0);
                    v.b = v.a;
                }
                buf0[2 * q] = v.a;
                buf0[2 * q + 1] = v.b;
            }
        }
        __syncthreads();
        T2* res = fft_lane<T2>(buf0, buf1, S, lt, TS, LF);
        if (colvalid) {
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int q = lt + h * TS;
                if (q < H) {
                    T2 X[2];
                    rfft_split<T>(res, S, q, pw[h], a.conj, X);
                    Pair<T2> o;
                    o.a = X[0];
                    o.b = X[1];
                    outp[chunk / 2 + q] = o;
                }
            }
        }
        __syncthreads();
    }
}

// Scaled gradients G = h grad u of the six triangles around interior node (i, j) from the values
// of u at the node and its neighbours, with the scaled gradient of the node's hat function on
// each: T_a(i,j) (-1,0), T_b(i,j) (0,-1), T_a(i-1,j) (1,-1), T_b(i,j-1) (-1,1),
// T_a(i-1,j-1) (0,1), T_b(i-1,j-1) (1,0); and the six triangle ids.
struct Six {
    double gx[6], gy[6];
    size_t tri[6];
};

__device__ __forceinline__ Six six_triangles(int n, int i, int j, double uc, double ue, double uw, double un,
                                             double us, double une, double usw) {
    Six t;
    t.gx[0] = ue - uc;   t.gy[0] = une - ue;    // T_a(i,j)
    t.gx[1] = une - un;  t.gy[1] = un - uc;     // T_b(i,j)
    t.gx[2] = uc - uw;   t.gy[2] = un - uc;     // T_a(i-1,j)
    t.gx[3] = ue - uc;   t.gy[3] = uc - us;     // T_b(i,j-1)
    t.gx[4] = us - usw;  t.gy[4] = uc - us;     // T_a(i-1,j-1)
    t.gx[5] = uc - uw;   t.gy[5] = uw - usw;    // T_b(i-1,j-1)
    const size_t c = (size_t)j * n + i;
    t.tri[0] = 2 * c;
    t.tri[1] = 2 * c + 1;
    t.tri[2] = 2 * (c - 1);
    t.tri[3] = 2 * (c - n) + 1;
    t.tri[4] = 2 * (c - n - 1);
    t.tri[5] = 2 * (c - n - 1) + 1;
    return t;
}

// K(u)_i = sum_T |T| nu_T grad u_T . grad phi_i = (1/2) sum_T nu_T G_T . g~_T with the law of each
// triangle's region (times theta), s^2 = n^2 |G|^2.
template <int LAW>
__device__ __forceinline__ double k_six(const Six& t, const FwdArgs& a, const double4* regp) {
    const int px[6] = {-1, 0, 1, -1, 0, 1};
    const int py[6] = {0, -1, -1, 1, 1, 0};
    double K = 0.0;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const double th = a.theta ? a.theta[t.tri[k]] : 1.0;
        const double s2 = a.n2 * (t.gx[k] * t.gx[k] + t.gy[k] * t.gy[k]);
        const double nu = th * law_nu<LAW>(regp[a.flags[t.tri[k]]], s2);
        K += nu * (t.gx[k] * px[k] + t.gy[k] * py[k]);
    }
    return 0.5 * K;
}

template <int LAW>
__global__ void __launch_bounds__(kBlock) k_apply_K(FwdArgs a, int nslices, double* ku) {
    size_t total = (size_t)nslices * a.nodes;
    const size_t sd = a.side;
    for (size_t id = blockIdx.x * (size_t)kBlock + threadIdx.x; id < total; id += (size_t)gridDim.x * kBlock) {
        size_t node = id % a.nodes;
        int i = (int)(node % sd), j = (int)(node / sd);
        if (!(i > 0 && j > 0 && i < a.n && j < a.n)) {
            ku[id] = 0.0;
            continue;
        }
        const double* u = a.U + id;
        // neighbours on the boundary are read as 0 (u = 0 there), whatever the field holds
        auto at = [&](int di, int dj) -> double {
            const int ii = i + di, jj = j + dj;
            return (ii > 0 && jj > 0 && ii < a.n && jj < a.n) ? u[(long)dj * (long)sd + di] : 0.0;
        };
        const Six t = six_triangles(a.n, i, j, u[0], at(1, 0), at(-1, 0), at(0, 1), at(0, -1), at(1, 1), at(-1, -1));
        ku[id] = k_six<LAW>(t, a, a.regp);
    }
}


int launch_forward(const Plan& p, char* ws, int mode, const double* Uw, void* out, double* rout, double* part,
                   hipStream_t st) {
    FwdArgs a;
    a.n = p.n;
    a.side = p.side;
    a.N = p.N;
    a.S = p.S;
    a.lgS = 0;
    while ((1 << a.lgS) < p.S) ++a.lgS;
    a.B = p.B;
    a.ST = p.ST;
    a.lgST = 0;
    while ((1 << a.lgST) < p.ST) ++a.lgST;
    a.regp = (const double4*)(ws + p.off_regp);
    a.remap = p.opt.xcd_remap;
    a.mode = mode;
    a.nodes = p.nodes;
    a.inv_tau = 1.0 / p.tau;
    a.n2 = (double)p.n * (double)p.n;
    a.U = Uw;
    a.F = p.prob.d_load ? (const double*)(ws + p.off_F) : nullptr;
    a.bload = (const double*)(ws + p.off_b);
    a.wave = (const double*)(ws + p.off_wave);
    a.mt = (const double*)(ws + p.lev[0].off_mt);
    a.flags = (const uint8_t*)(ws + p.off_flags);
    a.theta = p.prob.d_theta;
    a.rec = (const double*)(ws + p.off_rec);
    a.tw = ws + (p.fp32 ? p.off_tw32 : p.off_tw64);
    a.out = nullptr;
    a.rout = rout;
    a.part = part;
    // residual sweep: TS = min(S, 256) threads per column, KP = S / TS pairs per lane
    const int TS = p.S < kBlock ? p.S : kBlock;
    const int KP = p.S / TS;
    const int nb = kBlock / TS;
    const Geom& gf = p.g_fwd;
    a.ts = TS;
    a.nb = nb;
    a.col_groups = gf.col_groups;
    a.rows_per_chunk = gf.rows_per_chunk;
    size_t shm = (size_t)nb * kRowBatch * p.S * 4 * sizeof(double);
    if (shm < 2 * kBlock * sizeof(double)) shm = 2 * kBlock * sizeof(double);  // the norm reduction
    dim3 blk(nb * TS);
    bool uni = TS >= 64;
    void* rt = out ? (void*)(ws + p.off_P) : nullptr;  // R in solver precision, node-major
    tm_begin(p, KID_RESIDUAL, st);
    const int rk = mode == TM_SIGNAL ? RK_SIGNAL : (a.F ? RK_LOAD : RK_WAVE);
    // the law of the records (the field-copy mode reads none)
    const bool expcap = p.law == PT_NU_EXPCAP && rk != RK_SIGNAL;
    // residual spectrum in one pass: transform fused into the sweep (see k_residual); its
    // S/4 lanes per node must lie in one wavefront, so S <= 256
    if (out && !rout && rk != RK_SIGNAL && KP == 1 && p.S >= 4 && p.S <= 256) {
        a.out = out;
        shm += (size_t)p.N * p.elem;  // twiddle table
        auto fused = [&](auto t_, auto uni_, auto rk_, auto law_) {
            using TT = decltype(t_);
            constexpr bool U = decltype(uni_)::value;
            constexpr int G = decltype(rk_)::value, LW = decltype(law_)::value;
            hipLaunchKernelGGL((k_residual<TT, U, 1, G, true, LW>), dim3(gf.blocks), blk, shm, st, a, nullptr);
        };
        auto fused_law = [&](auto t_, auto uni_, auto rk_) {
            if (expcap) fused(t_, uni_, rk_, std::integral_constant<int, PT_NU_EXPCAP>());
            else fused(t_, uni_, rk_, std::integral_constant<int, PT_NU_RATIONAL>());
        };
        auto fused_rk = [&](auto t_, auto uni_) {
            if (rk == RK_LOAD) fused_law(t_, uni_, std::integral_constant<int, RK_LOAD>());
            else fused_law(t_, uni_, std::integral_constant<int, RK_WAVE>());
        };
        auto fused_t = [&](auto t_) {
            if (uni) fused_rk(t_, std::true_type());
            else fused_rk(t_, std::false_type());
        };
        if (p.fp32)
            fused_t(0.0f);
        else
            fused_t(0.0);
        tm_end(p, KID_RESIDUAL, st);
        return 0;
    }
    auto sweep = [&](auto t_, auto uni_, auto kp_, auto rk_, auto law_) {
        using TT = decltype(t_);
        constexpr bool U = decltype(uni_)::value;
        constexpr int K = decltype(kp_)::value, G = decltype(rk_)::value, LW = decltype(law_)::value;
        hipLaunchKernelGGL((k_residual<TT, U, K, G, false, LW>), dim3(gf.blocks), blk, shm, st, a, rt);
    };
    auto sweep_rk = [&](auto t_, auto uni_, auto kp_) {
        using RAT = std::integral_constant<int, PT_NU_RATIONAL>;
        using EXP = std::integral_constant<int, PT_NU_EXPCAP>;
        if (rk == RK_SIGNAL) sweep(t_, uni_, kp_, std::integral_constant<int, RK_SIGNAL>(), RAT());
        else if (rk == RK_LOAD) {
            if (expcap) sweep(t_, uni_, kp_, std::integral_constant<int, RK_LOAD>(), EXP());
            else sweep(t_, uni_, kp_, std::integral_constant<int, RK_LOAD>(), RAT());
        } else {
            if (expcap) sweep(t_, uni_, kp_, std::integral_constant<int, RK_WAVE>(), EXP());
            else sweep(t_, uni_, kp_, std::integral_constant<int, RK_WAVE>(), RAT());
        }
    };
    auto sweep_t = [&](auto t_) {
        if (KP == 2) sweep_rk(t_, std::true_type(), std::integral_constant<int, 2>());
        else if (uni) sweep_rk(t_, std::true_type(), std::integral_constant<int, 1>());
        else sweep_rk(t_, std::false_type(), std::integral_constant<int, 1>());
    };
    if (p.fp32)
        sweep_t(0.0f);
    else
        sweep_t(0.0);
    tm_end(p, KID_RESIDUAL, st);
    if (out) launch_rfft(p, ws, rt, out, 0, st);
    return 0;
}

void launch_rfft(const Plan& p, char* ws, const void* rt, void* out, int conj, hipStream_t st) {
    RfftArgs b;
    const Geom& g = p.g_team;
    b.n = p.n;
    b.side = p.side;
    b.N = p.N;
    b.S = p.S;
    b.ts = g.slot_chunk;
    b.nb = g.per_step;
    b.col_groups = g.col_groups;
    b.rows_per_chunk = g.rows_per_chunk;
    b.remap = p.opt.xcd_remap;
    b.B = p.B;
    b.ST = p.ST;
    b.conj = conj;
    b.rt = rt;
    b.tw = ws + (p.fp32 ? p.off_tw32 : p.off_tw64);
    b.out = out;
    size_t shm2 = (size_t)g.per_step * 2 * p.S * p.elem;
    dim3 blk2(g.per_step * g.slot_chunk);
    tm_begin(p, KID_RFFT, st);
    if (p.fp32)
        hipLaunchKernelGGL(k_rfft<float>, dim3(g.blocks), blk2, shm2, st, b);
    else
        hipLaunchKernelGGL(k_rfft<double>, dim3(g.blocks), blk2, shm2, st, b);
    tm_end(p, KID_RFFT, st);
}

// ---------------------------------------------------------------- norm reduction

// Norm partials of the residual sweep: partial p belongs to virtual workgroup p / nb, team
// p % nb, i.e. virtual column ((p / nb) % col_groups) nb + p % nb; workgroup x = instance b sums
// the partials of its columns in a fixed order into out2[2 b], out2[2 b + 1].
__global__ void __launch_bounds__(kBlock) k_reduce_norms(const double* part, int nparts, int nb, int col_groups,
                                                         int side, double* out2) {
    __shared__ double red[2][kBlock];
    const int b = blockIdx.x;
    double s0 = 0, s1 = 0;
    // partials q = threadIdx.x + kBlock t in order of t; the loads of kReduceBatch of them are
    // issued together (indexes past nparts clamped onto the first one, loaded and not added)
    for (int q = threadIdx.x; q < nparts; q += kBlock * kReduceBatch) {
        double2 v[kReduceBatch];
#pragma unroll
        for (int u = 0; u < kReduceBatch; ++u) {
            const int qq = q + u * kBlock < nparts ? q + u * kBlock : q;
            v[u] = ((const double2*)part)[qq];
        }
#pragma unroll
        for (int u = 0; u < kReduceBatch; ++u) {
            const int qq = q + u * kBlock;
            if (qq >= nparts) continue;
            const int vcol = ((qq / nb) % col_groups) * nb + qq % nb;
            if (vcol / side != b) continue;
            s0 += v[u].x;
            s1 += v[u].y;
        }
    }
    red[0][threadIdx.x] = s0;
    red[1][threadIdx.x] = s1;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out2[2 * b] = red[0][0];
        out2[2 * b + 1] = red[1][0];
    }
}

void launch_reduce_pairs(const Plan& p, const double* part, int nparts, double* out2, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_norms, dim3(1), dim3(kBlock), 0, st, part, nparts, 1, 1, p.side, out2);
}

void launch_reduce_norms(const Plan& p, char* ws, double* part, int flat, double* out2, hipStream_t st) {
    (void)ws;
    if (flat > 0) {  // one pair of partials per workgroup of a single-instance kernel
        launch_reduce_pairs(p, part, flat, out2, st);
        return;
    }
    const Geom& g = p.g_fwd;
    hipLaunchKernelGGL(k_reduce_norms, dim3(p.B), dim3(kBlock), 0, st, (const double*)part, g.blocks * g.per_step,
                       g.per_step, g.col_groups, p.side, out2);
}

// ---------------------------------------------------------------- inverse kernel

struct InvArgs {
    int n, side, N, S, ts, nb, col_groups, rows_per_chunk, remap, accumulate, B, ST, conj;
    size_t nodes;
    const void* xhat;     // T2 [nodes][S]
    const double* coef;   // double2 [S] generic scalars or null
    const void* tw;       // T2 [N]
    double* U;            // [nodes][N]
};

// Inverse packed real DFT of one node per team and row (the inverse of k_rfft), scaled by
// the per-slot coefficients, added to (ACC) or stored as the time series. The rows of a
// chunk are software-pipelined: the spectrum of row j+1 and the field of row j are loaded
// at the start of row j (on every path: indexes clamped to valid memory), so both overlap
// the transform of row j; the results of row j are stored after the loads of row j+1 are
// issued, so that no register reuse behind a store in flight stalls the next row. The field
// is read and written with streaming access: each value once per sweep (FP32 at 1024^2 x 512:
// 2.03 -> 1.86 ms per launch).
template <typename T, bool ACC>
__global__ void __launch_bounds__(kBlock) k_inverse(InvArgs a) {
    using T2 = typename Vec2<T>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T2* smem = (T2*)smem_raw;
    const int TS = a.ts, S = a.S, H = S / 2;
    const int lt = threadIdx.x % TS, team = threadIdx.x / TS;
    T2* buf0 = smem + (size_t)team * 2 * S;
    T2* buf1 = buf0 + S;
    const T2* tw = (const T2*)a.tw;
    const T invS = (T)1 / (T)S;
    const LaneFft<T2> LF = lane_fft_twiddles<T2>(tw, S, lt, TS);
    const int vb = virtual_block(a.remap);
    const SweepRange sr = sweep_range(vb, a.col_groups, a.nb, a.rows_per_chunk, a.side);
    const int vcol = sr.col0 + team;  // b (n+1) + i
    const bool valid = vcol < a.side * a.B;
    const int bi = valid ? vcol / a.side : 0, i = valid ? vcol - bi * a.side : 0;
    // per-lane constants of the slot pairs q = lt + h TS: twiddles and coefficients of slots 2q, 2q+1
    T2 pw[2][2];
    GS<T> cf[2][2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
        const int q = (lt + h * TS) < H ? lt + h * TS : 0;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            const int k = 2 * q + e;
            pw[h][e] = conj2(tw[k]);
            if (a.coef) {
                cf[h][e] = gs_from<T>(((const double2*)a.coef)[bi * S + k], k == 0);
            } else {
                cf[h][e].a = (T)1;
                cf[h][e].b = (T)0;
                cf[h][e].c = (T)1;
            }
        }
    }
    // slot / time-pair offset of (row j, column i, instance bi); rows past the chunk map onto
    // its last row (loaded, never used)
    auto chunk_of = [&](int j) -> size_t {
        const int jj = j < sr.row1 ? j : sr.row1 - 1;
        return ((size_t)jj * a.side + i) * a.ST + (size_t)bi * S;
    };
    constexpr int kMaxPer = 4;  // S / TS time pairs per lane (TS = S / 4, or 1 when S = 2)
    auto load_x = [&](int j, Pair<T2>* pv) {
        const Pair<T2>* xp = (const Pair<T2>*)a.xhat + chunk_of(j) / 2;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int q = lt + h * TS;
            pv[h] = xp[q < H ? q : H - 1];
        }
    };
    Pair<T2> pn[2];
    if (sr.row0 < sr.row1) load_x(sr.row0, pn);
    double2 op[kMaxPer];   // results of the previous row, stored one row late
    double2* up = nullptr;
    auto store_prev = [&]() {
        if (!up) return;
#pragma unroll
        for (int r = 0; r < kMaxPer; ++r) {
            const int m = lt + r * TS;
            if (m < S) nt_store(&up[m], op[r]);
        }
    };
    for (int j = sr.row0; j < sr.row1; ++j) {
        const bool interior = valid && i > 0 && j > 0 && i < a.n && j < a.n;
        const size_t chunk = chunk_of(j);
        Pair<T2> pv[2] = {pn[0], pn[1]};
        load_x(j + 1, pn);
        double2 uo[kMaxPer];
        double2* u2 = (double2*)a.U + chunk;
        if constexpr (ACC) {
#pragma unroll
            for (int r = 0; r < kMaxPer; ++r) {
                const int m = lt + r * TS;
                uo[r] = nt_load(&u2[m < S ? m : S - 1]);
            }
        }
        issue_fence();
        store_prev();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            consume(pv[h].a);
            consume(pv[h].b);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int q = lt + h * TS;
            if (q < H) {
                T2 v[2] = {mk2<T>(0, 0), mk2<T>(0, 0)};
                if (interior) {
                    v[0] = pv[h].a;
                    v[1] = pv[h].b;
#pragma unroll
                    for (int e = 0; e < 2; ++e) {
                        v[e] = gs_apply(cf[h][e], v[e]);
                        if (a.conj && 2 * q + e != 0) v[e] = conj2(v[e]);
                    }
                }
                buf0[2 * q] = v[0];
                buf0[2 * q + 1] = v[1];
            }
        }
        __syncthreads();
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int q = lt + h * TS;
            if (q < H) {
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const int k = 2 * q + e;
                    T2 Z;
                    if (k == 0) {
                        T2 p0 = buf0[0];
                        Z = mk2<T>((T)0.5 * (p0.x + p0.y), (T)0.5 * (p0.x - p0.y));
                    } else {
                        T2 xk = buf0[k], xs = conj2(buf0[S - k]);
                        T2 E = scale2((T)0.5, add2(xk, xs));
                        T2 O = cmul(scale2((T)0.5, sub2(xk, xs)), pw[h][e]);
                        Z = mk2<T>(E.x - O.y, E.y + O.x);  // E + i O
                    }
                    buf1[k] = conj2(Z);
                }
            }
        }
        __syncthreads();
        T2* res = fft_lane<T2>(buf1, buf0, S, lt, TS, LF);
        up = (interior || (valid && !ACC)) ? u2 : nullptr;
#pragma unroll
        for (int r = 0; r < kMaxPer; ++r) {
            const int m = lt + r * TS;
            double2 o = make_double2(0.0, 0.0);
            if (interior && m < S) {
                const T2 z = res[m];
                o.x = (double)(z.x * invS);
                o.y = (double)(-z.y * invS);
                if constexpr (ACC) {
                    o.x += uo[r].x;
                    o.y += uo[r].y;
                }
            }
            op[r] = o;
            if constexpr (ACC) consume(uo[r]);
        }
        __syncthreads();
    }
    store_prev();
}

void launch_inverse(const Plan& p, char* ws, const void* xhat, const double* coef, double* Uw, int accumulate,
                    hipStream_t st, int conj) {
    InvArgs a;
    const Geom& g = p.g_team;
    a.n = p.n;
    a.side = p.side;
    a.N = p.N;
    a.S = p.S;
    a.ts = g.slot_chunk;
    a.nb = g.per_step;
    a.col_groups = g.col_groups;
    a.rows_per_chunk = g.rows_per_chunk;
    a.remap = p.opt.xcd_remap;
    a.accumulate = accumulate;
    a.B = p.B;
    a.ST = p.ST;
    a.conj = conj;
    a.nodes = p.nodes;
    a.xhat = xhat;
    a.coef = coef;
    a.tw = ws + (p.fp32 ? p.off_tw32 : p.off_tw64);
    a.U = Uw;
    size_t shm = (size_t)g.per_step * 2 * p.S * p.elem;
    dim3 blk(g.per_step * g.slot_chunk);
    if (p.fp32) {
        if (accumulate)
            hipLaunchKernelGGL((k_inverse<float, true>), dim3(g.blocks), blk, shm, st, a);
        else
            hipLaunchKernelGGL((k_inverse<float, false>), dim3(g.blocks), blk, shm, st, a);
    } else {
        if (accumulate)
            hipLaunchKernelGGL((k_inverse<double, true>), dim3(g.blocks), blk, shm, st, a);
        else
            hipLaunchKernelGGL((k_inverse<double, false>), dim3(g.blocks), blk, shm, st, a);
    }
}

// ---------------------------------------------------------------- transposes

// dst[c][r] = src[r][c] for r < rows, c < cols; entries whose node index (the row
// index when node_is_row, else the column index) lies on the grid boundary are 0.
__global__ void __launch_bounds__(kBlock) k_transpose(const double* __restrict__ src, double* __restrict__ dst,
                                                      size_t rows, size_t cols, int n, int node_is_row) {
    __shared__ double tile[32][33];
    size_t tiles_c = (cols + 31) / 32;
    size_t r0 = (blockIdx.x / tiles_c) * 32, c0 = (blockIdx.x % tiles_c) * 32;
    int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
    int side = n + 1;
    for (int k = ty; k < 32; k += 8) {
        size_t r = r0 + k, c = c0 + tx;
        double v = 0.0;
        if (r < rows && c < cols) {
            size_t node = node_is_row ? r : c;
            int i = (int)(node % side), j = (int)(node / side);
            bool interior = i > 0 && j > 0 && i < n && j < n;
            v = interior ? src[r * cols + c] : 0.0;
        }
        tile[k][tx] = v;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        size_t c = c0 + k, r = r0 + tx;
        if (r < rows && c < cols) dst[c * rows + r] = tile[tx][k];
    }
}

static unsigned transpose_grid(size_t rows, size_t cols) {
    return (unsigned)(((rows + 31) / 32) * ((cols + 31) / 32));
}

void launch_transpose_in(const Plan& p, const double* src, double* dst, hipStream_t st) {
    size_t rows = (size_t)p.B * p.N, cols = p.nodes;
    hipLaunchKernelGGL(k_transpose, dim3(transpose_grid(rows, cols)), dim3(kBlock), 0, st, src, dst, rows, cols,
                       p.n, 0);
}

void launch_transpose_out(const Plan& p, const double* src, double* dst, hipStream_t st) {
    size_t rows = p.nodes, cols = (size_t)p.B * p.N;
    hipLaunchKernelGGL(k_transpose, dim3(transpose_grid(rows, cols)), dim3(kBlock), 0, st, src, dst, rows, cols,
                       p.n, 1);
}

// ---------------------------------------------------------------- K(u) on slices

void launch_apply_K(const Plan& p, char* ws, const double* u, double* ku, int nslices, hipStream_t st) {
    FwdArgs a = {};
    a.n = p.n;
    a.side = p.side;
    a.nodes = p.nodes;
    a.n2 = (double)p.n * (double)p.n;
    a.regp = (const double4*)(ws + p.off_regp);
    a.U = u;
    a.flags = (const uint8_t*)(ws + p.off_flags);
    a.theta = p.prob.d_theta;
    size_t total = (size_t)nslices * p.nodes;
    size_t g = (total + kBlock - 1) / kBlock;
    if (g > 65536) g = 65536;
    if (p.law == PT_NU_EXPCAP)
        hipLaunchKernelGGL(k_apply_K<PT_NU_EXPCAP>, dim3((unsigned)g), dim3(kBlock), 0, st, a, nslices, ku);
    else
        hipLaunchKernelGGL(k_apply_K<PT_NU_RATIONAL>, dim3((unsigned)g), dim3(kBlock), 0, st, a, nslices, ku);
}

}  // namespace pt
