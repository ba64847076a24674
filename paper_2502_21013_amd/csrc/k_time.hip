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
#include "pt_device.h"

namespace pt {

// ---------------------------------------------------------------- in-LDS complex FFT

// Forward (unnormalised) complex DFT of length S of the team's buffer a, Stockham
// radix-4 stages and one radix-2 stage when log2 S is odd; b is scratch. tw[k] =
// exp(-2 pi i k / N) for k < N (so exp(-2 pi i m / S) = tw[2 m]). Every thread of the
// workgroup must call it (it synchronises the workgroup). Returns the result buffer.
template <typename T2>
__device__ T2* fft_team(T2* a, T2* b, int S, int lt, int TS, const T2* __restrict__ tw) {
    int Ns = 1;
    const int Q = S >> 2;
    while (Ns * 4 <= S) {
        for (int j = lt; j < Q; j += TS) {
            int k = j & (Ns - 1);
            T2 v0 = a[j], v1 = a[j + Q], v2 = a[j + 2 * Q], v3 = a[j + 3 * Q];
            if (Ns > 1) {
                int st = S / (2 * Ns);
                v1 = cmul(v1, tw[k * st]);
                v2 = cmul(v2, tw[2 * k * st]);
                v3 = cmul(v3, tw[3 * k * st]);
            }
            T2 t0 = add2(v0, v2), t1 = sub2(v0, v2), t2 = add2(v1, v3), t3 = mul_mi(sub2(v1, v3));
            int idx = (j / Ns) * Ns * 4 + k;
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
        for (int j = lt; j < H; j += TS) {
            int k = j & (Ns - 1);
            T2 v0 = a[j];
            T2 v1 = cmul(a[j + H], tw[k * S / Ns]);
            int idx = (j / Ns) * Ns * 2 + k;
            b[idx] = add2(v0, v1);
            b[idx + Ns] = sub2(v0, v1);
        }
        __syncthreads();
        T2* t = a;
        a = b;
        b = t;
    }
    return a;
}

// ---------------------------------------------------------------- forward kernel

struct FwdArgs {
    int n, side, N, S, ts, nb, steps, remap, mode;
    size_t nodes;
    double inv_tau, n2;
    double nu_a, nu_b, nu_out;
    const double* U;       // [nodes][N]
    const double* F;       // [nodes][N] explicit load or null
    const double* bload;   // [nodes]
    const double* wave;    // [N]
    const double* mt;      // [4][nodes]
    const uint8_t* flags;  // [2 n^2]
    const double* theta;   // [2 n^2] or null
    const void* tw;        // T2 [N]
    void* out;             // T2 [nodes][S] or null
    double* rout;          // [nodes][N] or null
    double* part;          // [gridDim.x][2]
};

__device__ __forceinline__ double nu_tri(double gx, double gy, const FwdArgs& a, bool iron, double th) {
    if (!iron) return th * a.nu_out;
    double s2 = a.n2 * (gx * gx + gy * gy);
    return th * (a.nu_a + a.nu_b * s2 / (1.0 + s2));
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_forward(FwdArgs a) {
    using T2 = typename Vec2<T>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T2* smem = (T2*)smem_raw;
    const int TS = a.ts, S = a.S, N = a.N;
    const int lt = threadIdx.x % TS, team = threadIdx.x / TS;
    T2* buf0 = smem + (size_t)team * 2 * S;
    T2* buf1 = buf0 + S;
    T* rb = (T*)buf0;
    const T2* tw = (const T2*)a.tw;
    const int vb = virtual_block(a.remap);
    double rr = 0.0, ff = 0.0;
    for (int step = 0; step < a.steps; ++step) {
        size_t node = ((size_t)vb * a.steps + step) * a.nb + team;
        bool valid = node < a.nodes;
        int i = valid ? (int)(node % a.side) : 0, j = valid ? (int)(node / a.side) : 0;
        bool interior = valid && i > 0 && j > 0 && i < a.n && j < a.n;
        if (interior) {
            const size_t nodes = a.nodes;
            const size_t sd = (size_t)a.side;
            const double* U = a.U + node * N;
            const long sN = (long)sd * N;
            double mc = 0, me = 0, mw = 0, mn = 0, ms = 0, mne = 0, msw = 0;
            bool mass = false;
            if (a.mode == TM_RESIDUAL) {
                mc = a.mt[node];
                me = a.mt[nodes + node];
                mw = a.mt[nodes + node - 1];
                mn = a.mt[2 * nodes + node];
                ms = a.mt[2 * nodes + node - sd];
                mne = a.mt[3 * nodes + node];
                msw = a.mt[3 * nodes + node - sd - 1];
                mass = (mc != 0.0) || (me != 0.0) || (mw != 0.0) || (mn != 0.0) || (ms != 0.0) || (mne != 0.0) ||
                       (msw != 0.0);
            }
            // the six triangles around node (i, j)
            size_t c_ij = (size_t)j * a.n + i, c_w = c_ij - 1, c_s = c_ij - a.n, c_sw = c_ij - a.n - 1;
            bool ir1 = a.flags[2 * c_ij] & 1, ir2 = a.flags[2 * c_ij + 1] & 1, ir3 = a.flags[2 * c_w] & 1,
                 ir4 = a.flags[2 * c_s + 1] & 1, ir5 = a.flags[2 * c_sw] & 1, ir6 = a.flags[2 * c_sw + 1] & 1;
            double th1 = 1, th2 = 1, th3 = 1, th4 = 1, th5 = 1, th6 = 1;
            if (a.theta) {
                th1 = a.theta[2 * c_ij];
                th2 = a.theta[2 * c_ij + 1];
                th3 = a.theta[2 * c_w];
                th4 = a.theta[2 * c_s + 1];
                th5 = a.theta[2 * c_sw];
                th6 = a.theta[2 * c_sw + 1];
            }
            double bl = a.bload[node];
            for (int q = lt; q < N; q += TS) {
                double R;
                if (a.mode == TM_RESIDUAL) {
                    double uc = U[q], ue = U[N + q], uw = U[q - N], un = U[sN + q], us = U[q - sN];
                    double une = U[sN + N + q], usw = U[q - sN - N];
                    double g1x = ue - uc, g1y = une - ue;      // T_a(i,j)
                    double g2x = une - un, g2y = un - uc;      // T_b(i,j)
                    double g3x = uc - uw, g3y = un - uc;       // T_a(i-1,j)
                    double g4x = ue - uc, g4y = uc - us;       // T_b(i,j-1)
                    double g5x = us - usw, g5y = uc - us;      // T_a(i-1,j-1)
                    double g6x = uc - uw, g6y = uw - usw;      // T_b(i-1,j-1)
                    double K = nu_tri(g1x, g1y, a, ir1, th1) * (-g1x) + nu_tri(g2x, g2y, a, ir2, th2) * (-g2y) +
                               nu_tri(g3x, g3y, a, ir3, th3) * (g3x - g3y) +
                               nu_tri(g4x, g4y, a, ir4, th4) * (g4y - g4x) + nu_tri(g5x, g5y, a, ir5, th5) * g5y +
                               nu_tri(g6x, g6y, a, ir6, th6) * g6x;
                    K *= 0.5;
                    double f = a.F ? a.F[node * N + q] : bl * a.wave[q];
                    double Md = 0.0;
                    if (mass) {
                        int qm = (q == 0) ? N - 1 : q - 1;
                        Md = mc * (uc - U[qm]) + me * (ue - U[N + qm]) + mw * (uw - U[qm - N]) +
                             mn * (un - U[sN + qm]) + ms * (us - U[qm - sN]) + mne * (une - U[sN + N + qm]) +
                             msw * (usw - U[qm - sN - N]);
                    }
                    R = f - Md * a.inv_tau - K;
                    ff += f * f;
                } else {
                    R = U[q];
                }
                rr += R * R;
                rb[q] = (T)R;
                if (a.rout) a.rout[node * N + q] = R;
            }
        } else {
            for (int q = lt; q < N; q += TS) rb[q] = (T)0;
            if (valid && a.rout)
                for (int q = lt; q < N; q += TS) a.rout[node * N + q] = 0.0;
        }
        __syncthreads();
        if (a.out) {
            T2* res = fft_team<T2>(buf0, buf1, S, lt, TS, tw);
            if (valid) {
                T2* out = (T2*)a.out + node * S;
                for (int k = lt; k < S; k += TS) {
                    T2 X;
                    if (k == 0) {
                        T2 z0 = res[0];
                        X = mk2<T>(z0.x + z0.y, z0.x - z0.y);
                    } else {
                        T2 zk = res[k], zc = conj2(res[S - k]);
                        T2 E = scale2((T)0.5, add2(zk, zc));
                        T2 O = scale2((T)0.5, mul_mi(sub2(zk, zc)));
                        X = add2(E, cmul(tw[k], O));
                    }
                    out[k] = X;
                }
            }
        }
        __syncthreads();
    }
    // workgroup reduction of the norm partials (fixed order)
    __shared__ double red[2][kBlock];
    red[0][threadIdx.x] = rr;
    red[1][threadIdx.x] = ff;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            red[0][threadIdx.x] += red[0][threadIdx.x + w];
            red[1][threadIdx.x] += red[1][threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0 && a.part) {
        a.part[2 * blockIdx.x] = red[0][0];
        a.part[2 * blockIdx.x + 1] = red[1][0];
    }
}

void launch_forward(const Plan& p, char* ws, int mode, const double* Uw, void* out, double* rout, double* part,
                    hipStream_t st) {
    FwdArgs a;
    const Geom& g = p.g_team;
    a.n = p.n;
    a.side = p.side;
    a.N = p.N;
    a.S = p.S;
    a.ts = g.slot_chunk;
    a.nb = g.per_step;
    a.steps = g.steps;
    a.remap = p.opt.xcd_remap;
    a.mode = mode;
    a.nodes = p.nodes;
    a.inv_tau = 1.0 / p.tau;
    a.n2 = (double)p.n * (double)p.n;
    a.nu_a = p.prob.nu_a;
    a.nu_b = p.prob.nu_b;
    a.nu_out = p.prob.nu_out;
    a.U = Uw;
    a.F = p.prob.d_load ? (const double*)(ws + p.off_F) : nullptr;
    a.bload = (const double*)(ws + p.off_b);
    a.wave = (const double*)(ws + p.off_wave);
    a.mt = (const double*)(ws + p.lev[0].off_mt);
    a.flags = (const uint8_t*)(ws + p.off_flags);
    a.theta = p.prob.d_theta;
    a.tw = ws + (p.fp32 ? p.off_tw32 : p.off_tw64);
    a.out = out;
    a.rout = rout;
    a.part = part;
    size_t shm = (size_t)g.per_step * 2 * p.S * p.elem;
    if (p.fp32)
        hipLaunchKernelGGL(k_forward<float>, dim3(g.blocks), dim3(kBlock), shm, st, a);
    else
        hipLaunchKernelGGL(k_forward<double>, dim3(g.blocks), dim3(kBlock), shm, st, a);
}

// ---------------------------------------------------------------- norm reduction

__global__ void __launch_bounds__(kBlock) k_reduce_norms(const double* part, int nparts, double* out2) {
    __shared__ double red[2][kBlock];
    double s0 = 0, s1 = 0;
    for (int b = threadIdx.x; b < nparts; b += kBlock) {
        s0 += part[2 * b];
        s1 += part[2 * b + 1];
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
        out2[0] = red[0][0];
        out2[1] = red[1][0];
    }
}

void launch_reduce_norms(const Plan& p, char* ws, double* part, int nparts, double* out2, hipStream_t st) {
    (void)p;
    (void)ws;
    hipLaunchKernelGGL(k_reduce_norms, dim3(1), dim3(kBlock), 0, st, (const double*)part, nparts, out2);
}

// ---------------------------------------------------------------- inverse kernel

struct InvArgs {
    int n, side, N, S, ts, nb, steps, remap, accumulate;
    size_t nodes;
    const void* xhat;     // T2 [nodes][S]
    const double* coef;   // double2 [S] generic scalars or null
    const void* tw;       // T2 [N]
    double* U;            // [nodes][N]
};

template <typename T>
__global__ void __launch_bounds__(kBlock) k_inverse(InvArgs a) {
    using T2 = typename Vec2<T>::type;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T2* smem = (T2*)smem_raw;
    const int TS = a.ts, S = a.S, N = a.N;
    const int lt = threadIdx.x % TS, team = threadIdx.x / TS;
    T2* buf0 = smem + (size_t)team * 2 * S;
    T2* buf1 = buf0 + S;
    const T2* tw = (const T2*)a.tw;
    const T invS = (T)1 / (T)S;
    const int vb = virtual_block(a.remap);
    for (int step = 0; step < a.steps; ++step) {
        size_t node = ((size_t)vb * a.steps + step) * a.nb + team;
        bool valid = node < a.nodes;
        int i = valid ? (int)(node % a.side) : 0, j = valid ? (int)(node / a.side) : 0;
        bool interior = valid && i > 0 && j > 0 && i < a.n && j < a.n;
        const T2* x = (const T2*)a.xhat + node * S;
        for (int k = lt; k < S; k += TS) {
            T2 v = mk2<T>(0, 0);
            if (interior) {
                v = x[k];
                if (a.coef) {
                    double2 c = ((const double2*)a.coef)[k];
                    v = gs_apply(gs_from<T>(c, k == 0), v);
                }
            }
            buf0[k] = v;
        }
        __syncthreads();
        for (int k = lt; k < S; k += TS) {
            T2 Z;
            if (k == 0) {
                T2 p0 = buf0[0];
                Z = mk2<T>((T)0.5 * (p0.x + p0.y), (T)0.5 * (p0.x - p0.y));
            } else {
                T2 xk = buf0[k], xs = conj2(buf0[S - k]);
                T2 E = scale2((T)0.5, add2(xk, xs));
                T2 O = cmul(scale2((T)0.5, sub2(xk, xs)), conj2(tw[k]));
                Z = mk2<T>(E.x - O.y, E.y + O.x);  // E + i O
            }
            buf1[k] = conj2(Z);
        }
        __syncthreads();
        T2* res = fft_team<T2>(buf1, buf0, S, lt, TS, tw);
        if (interior) {
            double2* u2 = (double2*)(a.U + node * N);
            for (int m = lt; m < S; m += TS) {
                T2 z = res[m];
                double x0 = (double)(z.x * invS), x1 = (double)(-z.y * invS);
                double2 o;
                if (a.accumulate) {
                    o = u2[m];
                    o.x += x0;
                    o.y += x1;
                } else {
                    o.x = x0;
                    o.y = x1;
                }
                u2[m] = o;
            }
        } else if (valid && !a.accumulate) {
            double2* u2 = (double2*)(a.U + node * N);
            for (int m = lt; m < S; m += TS) u2[m] = make_double2(0.0, 0.0);
        }
        __syncthreads();
    }
}

void launch_inverse(const Plan& p, char* ws, const void* xhat, const double* coef, double* Uw, int accumulate,
                    hipStream_t st) {
    InvArgs a;
    const Geom& g = p.g_team;
    a.n = p.n;
    a.side = p.side;
    a.N = p.N;
    a.S = p.S;
    a.ts = g.slot_chunk;
    a.nb = g.per_step;
    a.steps = g.steps;
    a.remap = p.opt.xcd_remap;
    a.accumulate = accumulate;
    a.nodes = p.nodes;
    a.xhat = xhat;
    a.coef = coef;
    a.tw = ws + (p.fp32 ? p.off_tw32 : p.off_tw64);
    a.U = Uw;
    size_t shm = (size_t)g.per_step * 2 * p.S * p.elem;
    if (p.fp32)
        hipLaunchKernelGGL(k_inverse<float>, dim3(g.blocks), dim3(kBlock), shm, st, a);
    else
        hipLaunchKernelGGL(k_inverse<double>, dim3(g.blocks), dim3(kBlock), shm, st, a);
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
    size_t rows = p.N, cols = p.nodes;
    hipLaunchKernelGGL(k_transpose, dim3(transpose_grid(rows, cols)), dim3(kBlock), 0, st, src, dst, rows, cols,
                       p.n, 0);
}

void launch_transpose_out(const Plan& p, const double* src, double* dst, hipStream_t st) {
    size_t rows = p.nodes, cols = p.N;
    hipLaunchKernelGGL(k_transpose, dim3(transpose_grid(rows, cols)), dim3(kBlock), 0, st, src, dst, rows, cols,
                       p.n, 1);
}

// ---------------------------------------------------------------- K(u) on slices

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
        double uc = u[0], ue = u[1], uw = u[-1], un = u[sd], us = u[-(long)sd], une = u[sd + 1],
               usw = u[-(long)sd - 1];
        size_t c_ij = (size_t)j * a.n + i, c_w = c_ij - 1, c_s = c_ij - a.n, c_sw = c_ij - a.n - 1;
        bool ir1 = a.flags[2 * c_ij] & 1, ir2 = a.flags[2 * c_ij + 1] & 1, ir3 = a.flags[2 * c_w] & 1,
             ir4 = a.flags[2 * c_s + 1] & 1, ir5 = a.flags[2 * c_sw] & 1, ir6 = a.flags[2 * c_sw + 1] & 1;
        double th1 = 1, th2 = 1, th3 = 1, th4 = 1, th5 = 1, th6 = 1;
        if (a.theta) {
            th1 = a.theta[2 * c_ij];
            th2 = a.theta[2 * c_ij + 1];
            th3 = a.theta[2 * c_w];
            th4 = a.theta[2 * c_s + 1];
            th5 = a.theta[2 * c_sw];
            th6 = a.theta[2 * c_sw + 1];
        }
        double g1x = ue - uc, g1y = une - ue;
        double g2x = une - un, g2y = un - uc;
        double g3x = uc - uw, g3y = un - uc;
        double g4x = ue - uc, g4y = uc - us;
        double g5x = us - usw, g5y = uc - us;
        double g6x = uc - uw, g6y = uw - usw;
        double K = nu_tri(g1x, g1y, a, ir1, th1) * (-g1x) + nu_tri(g2x, g2y, a, ir2, th2) * (-g2y) +
                   nu_tri(g3x, g3y, a, ir3, th3) * (g3x - g3y) + nu_tri(g4x, g4y, a, ir4, th4) * (g4y - g4x) +
                   nu_tri(g5x, g5y, a, ir5, th5) * g5y + nu_tri(g6x, g6y, a, ir6, th6) * g6x;
        ku[id] = 0.5 * K;
    }
}

void launch_apply_K(const Plan& p, char* ws, const double* u, double* ku, int nslices, hipStream_t st) {
    FwdArgs a = {};
    a.n = p.n;
    a.side = p.side;
    a.nodes = p.nodes;
    a.n2 = (double)p.n * (double)p.n;
    a.nu_a = p.prob.nu_a;
    a.nu_b = p.prob.nu_b;
    a.nu_out = p.prob.nu_out;
    a.U = u;
    a.flags = (const uint8_t*)(ws + p.off_flags);
    a.theta = p.prob.d_theta;
    size_t total = (size_t)nslices * p.nodes;
    size_t g = (total + kBlock - 1) / kBlock;
    if (g > 65536) g = 65536;
    hipLaunchKernelGGL(k_apply_K, dim3((unsigned)g), dim3(kBlock), 0, st, a, nslices, ku);
}

}  // namespace pt
