// C ABI of the solver: plan validation, workspace layout, the outer fixed-point loop
// (Sec. 3, eqs. (iter1)-(iter2), correction form) and the component entry points.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <atomic>
#include <chrono>
#include <mutex>
#include <thread>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "pt_internal.h"

namespace pt {

static thread_local std::string g_last_error;

static pt_status fail(pt_status s, const std::string& msg) {
    g_last_error = msg;
    return s;
}

// Diagnostic output on stderr, chosen by the environment variable PT_LOG (read once):
// 0 or unset: none; 1: one line per plan and per solve (sizes, status, steps, residual, time);
// 2: also the relative residual at every check of the outer loop.
static int log_level() {
    static const int level = [] {
        const char* e = std::getenv("PT_LOG");
        return e ? std::atoi(e) : 0;
    }();
    return level;
}

#define PT_LOG(lvl, ...)                              \
    do {                                              \
        if (log_level() >= (lvl)) {                   \
            std::fprintf(stderr, "[ptsolve] " __VA_ARGS__); \
            std::fputc('\n', stderr);                 \
        }                                             \
    } while (0)

#define PT_HIP(call)                                                                               \
    do {                                                                                           \
        hipError_t e_ = (call);                                                                    \
        if (e_ != hipSuccess)                                                                      \
            return fail(PT_ERR_HIP, std::string(#call) + ": " + hipGetErrorString(e_));            \
    } while (0)

// ---------------------------------------------------------------- per-kernel event timer

static void tm_flush(const Plan& p) {
    Timer* t = p.tm;
    if (!t || !t->on || t->used == 0) return;
    hipEventSynchronize(t->ev[2 * t->used - 1]);
    for (int i = 0; i < t->used; ++i) {
        float ms = 0.f;
        hipEventElapsedTime(&ms, t->ev[2 * i], t->ev[2 * i + 1]);
        t->ms[t->kid[i]] += ms;
        t->cnt[t->kid[i]] += 1;
    }
    t->used = 0;
}

void tm_begin(const Plan& p, int kid, hipStream_t st) {
    Timer* t = p.tm;
    if (!t || !t->on || !((t->mask >> kid) & 1u)) return;
    if (t->used == Timer::kCap) tm_flush(p);
    hipEventRecord(t->ev[2 * t->used], st);
}

void tm_end(const Plan& p, int kid, hipStream_t st) {
    Timer* t = p.tm;
    if (!t || !t->on || !((t->mask >> kid) & 1u)) return;
    hipEventRecord(t->ev[2 * t->used + 1], st);
    t->kid[t->used] = kid;
    t->used += 1;
}

#define TM(kid, stmt)              \
    do {                           \
        tm_begin(p, (kid), st);    \
        stmt;                      \
        tm_end(p, (kid), st);      \
    } while (0)

static bool is_pow2(long v) { return v > 0 && (v & (v - 1)) == 0; }
static size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

static void sweep_geom(Geom& g, int side, int target_blocks, int cols = 0) {
    if (cols <= 0) cols = side;
    g.col_groups = (cols + g.per_step - 1) / g.per_step;
    int nch = target_blocks / (g.col_groups * g.chunks);
    if (nch < 1) nch = 1;
    if (nch > side) nch = side;
    g.rows_per_chunk = (side + nch - 1) / nch;
    nch = (side + g.rows_per_chunk - 1) / g.rows_per_chunk;
    size_t blocks = (size_t)g.col_groups * nch;
    blocks = (blocks + kNumXcd - 1) / kNumXcd * kNumXcd;
    g.blocks = (int)blocks;
}

Geom slot_geom(int side, int S, int V, int target_blocks, int cols, int max_chunk) {
    // S slots per node, V slots per lane: a workgroup row of slot_chunk <= max_chunk lanes
    // covers slot_chunk V slots; per_step column units (cols of them, default: the grid's
    // columns) per workgroup
    Geom g;
    const int lanes = S / V;
    g.slot_chunk = lanes < max_chunk ? lanes : max_chunk;
    g.per_step = kBlock / g.slot_chunk;
    g.chunks = lanes / g.slot_chunk;
    sweep_geom(g, side, target_blocks, cols);
    return g;
}

Geom team_geom(int side, int S, int B, int target_blocks) {
    Geom g;
    // S/4 threads per node (one radix-4 butterfly per thread and stage) and at least one
    // wavefront per workgroup: 64 / (S/4) nodes per workgroup when S < 256, one node
    // (one or two wavefronts) otherwise.
    int ts = S / 4;
    if (ts < 1) ts = 1;
    if (ts > kBlock) ts = kBlock;
    g.slot_chunk = ts;
    g.per_step = ts >= 64 ? 1 : 64 / ts;
    g.chunks = 1;
    sweep_geom(g, side, target_blocks, side * B);
    return g;
}

Geom fwd_geom(int side, int S, int B, int target_blocks) {
    Geom g;
    int ts = S < kBlock ? S : kBlock;
    g.slot_chunk = ts;
    g.per_step = kBlock / ts;
    g.chunks = 1;
    sweep_geom(g, side, target_blocks, side * B);
    return g;
}

static bool rect_ok(const pt_rect& r) {
    return std::isfinite(r.x0) && std::isfinite(r.y0) && std::isfinite(r.x1) && std::isfinite(r.y1);
}

static pt_status validate(const pt_problem* pr, const pt_options* o) {
    if (!pr || !o) return fail(PT_ERR_INVALID, "problem and options must not be NULL");
    if (!is_pow2(pr->n) || pr->n < 4 || pr->n > 4096) return fail(PT_ERR_INVALID, "n must be a power of two in [4, 4096]");
    if (!is_pow2(pr->N) || pr->N < 4 || pr->N > 1024) return fail(PT_ERR_INVALID, "N must be a power of two in [4, 1024]");
    if (!(pr->T > 0) || !std::isfinite(pr->T)) return fail(PT_ERR_INVALID, "T must be positive and finite");
    if (!(pr->sigma_in >= 0) || !std::isfinite(pr->sigma_in)) return fail(PT_ERR_INVALID, "sigma_in must be >= 0");
    if (!(pr->nu_max > 0) || !std::isfinite(pr->nu_max)) return fail(PT_ERR_INVALID, "nu_max must be positive");
    if (!std::isfinite(pr->nu_a) || !std::isfinite(pr->nu_b) || !std::isfinite(pr->nu_out) || !std::isfinite(pr->J0))
        return fail(PT_ERR_INVALID, "material and source parameters must be finite");
    if (!(pr->nu_a > 0) || !(pr->nu_a + pr->nu_b > 0) || !(pr->nu_out > 0))
        return fail(PT_ERR_INVALID, "the reluctivity must stay positive (nu_a > 0, nu_a + nu_b > 0, nu_out > 0)");
    if (!rect_ok(pr->sigma_rect) || !rect_ok(pr->nu_rect) || !rect_ok(pr->coil_rect))
        return fail(PT_ERR_INVALID, "rectangles must be finite");
    if (pr->waveform != PT_WAVE_SIN && pr->waveform != PT_WAVE_COS) return fail(PT_ERR_INVALID, "unknown waveform");
    if (pr->law != PT_NU_RATIONAL && pr->law != PT_NU_EXPCAP) return fail(PT_ERR_INVALID, "unknown reluctivity law");
    if (pr->nregions < 0 || pr->nregions > kMaxRegions) return fail(PT_ERR_INVALID, "nregions must be in [0, 16]");
    if (pr->nregions == 0 && pr->law != PT_NU_RATIONAL)
        return fail(PT_ERR_INVALID, "the exp-capped law needs region mode (nregions > 0)");
    if (pr->nregions > 0) {
        if (!pr->d_region || !pr->regions) return fail(PT_ERR_INVALID, "region mode needs d_region and regions");
        if (pr->d_sigma) return fail(PT_ERR_INVALID, "region mode takes the conductivity from the regions (d_sigma NULL)");
        for (int r = 0; r < pr->nregions; ++r) {
            const pt_region& g = pr->regions[r];
            if (!std::isfinite(g.sigma) || !std::isfinite(g.a) || !std::isfinite(g.b) || !std::isfinite(g.c) ||
                !std::isfinite(g.d) || !std::isfinite(g.j) || !(g.sigma >= 0) || !std::isfinite(g.nu_hat) ||
                !(g.nu_hat >= 0))
                return fail(PT_ERR_INVALID, "region " + std::to_string(r) +
                                                ": parameters must be finite, sigma >= 0 and nu_hat >= 0");
            const bool ok = pr->law == PT_NU_RATIONAL ? (g.a > 0 && g.a + g.b > 0)
                                                      : (g.a >= 0 && g.b >= 0 && g.c >= 1 && g.d > 0);
            if (!ok) return fail(PT_ERR_INVALID, "region " + std::to_string(r) + ": the law's parameters are out of range");
        }
    }
    if (!(o->tol > 0) || !std::isfinite(o->tol)) return fail(PT_ERR_INVALID, "tol must be positive");
    if (o->max_outer < 1) return fail(PT_ERR_INVALID, "max_outer must be >= 1");
    if (o->check_every < 1) return fail(PT_ERR_INVALID, "check_every must be >= 1");
    if (o->precision != PT_FP64 && o->precision != PT_FP32_REFINE) return fail(PT_ERR_INVALID, "unknown precision");
    if (o->inner != PT_INNER_GALERKIN1 && o->inner != PT_INNER_COCG) return fail(PT_ERR_INVALID, "unknown inner method");
    if (o->inner_iters < 1 || o->inner_iters > 64) return fail(PT_ERR_INVALID, "inner_iters must be in [1, 64]");
    if (o->vc_sweeps != 1) return fail(PT_ERR_INVALID, "vc_sweeps must be 1 (fused smoothing sweeps)");
    if (o->vc_cycle != PT_VC_DEFAULT && o->vc_cycle != PT_VC_V11 && o->vc_cycle != PT_VC_V01)
        return fail(PT_ERR_INVALID, "unknown vc_cycle");
    if (o->timing_mask < 0 || o->timing_mask >= (1 << KID_COUNT))
        return fail(PT_ERR_INVALID, "timing_mask has bits beyond the kernel classes");
    if (o->vc_cycle == PT_VC_V01 && o->inner == PT_INNER_COCG)
        return fail(PT_ERR_INVALID, "COCG needs the symmetric V(1,1) cycle (vc_cycle PT_VC_V11)");
    if (!(o->inner_rtol >= 0 && o->inner_rtol < 1)) return fail(PT_ERR_INVALID, "inner_rtol must be in [0, 1)");
    if (!(o->breakdown_tol >= 0) || !std::isfinite(o->breakdown_tol))
        return fail(PT_ERR_INVALID, "breakdown_tol must be finite and >= 0");
    if (!(o->vc_omega > 0 && o->vc_omega < 1)) return fail(PT_ERR_INVALID, "vc_omega must be in (0, 1)");
    if (o->adjoint != 0 && o->adjoint != 1) return fail(PT_ERR_INVALID, "adjoint must be 0 or 1");
    if (o->init_static != 0 && o->init_static != 1) return fail(PT_ERR_INVALID, "init_static must be 0 or 1");
    if (o->krylov_dim < 0 || o->krylov_dim > 64) return fail(PT_ERR_INVALID, "krylov_dim must be in [0, 64]");
    if (o->krylov_dim > 0 && (!(o->forcing > 0 && o->forcing < 1) || o->max_krylov < 1))
        return fail(PT_ERR_INVALID, "forcing must be in (0, 1) and max_krylov >= 1");
    if (o->init_static && (!(o->init_tol > 0) || !std::isfinite(o->init_tol)))
        return fail(PT_ERR_INVALID, "init_tol must be positive");
    if (o->init_static && o->use_initial_guess)
        return fail(PT_ERR_INVALID, "init_static and use_initial_guess cannot be combined");
    for (int32_t g : {o->grid_slot, o->grid_team, o->grid_restrict, o->grid_up, o->grid_matvec})
        if (g < 0 || (g > 0 && g < 8) || g > (1 << 22))
            return fail(PT_ERR_INVALID, "grid targets (grid_slot, grid_team, grid_restrict, grid_up, grid_matvec) "
                                        "must be 0 or in [8, 4194304]");
    if (!(o->diverge_factor >= 0) || !std::isfinite(o->diverge_factor))
        return fail(PT_ERR_INVALID, "diverge_factor must be >= 0");
    return PT_OK;
}

// A batch shares the grid, the period, the conductivity (so M and the multigrid
// hierarchy) and nu_max (so Khat); the reluctivity law, the iron region and the source
// may differ per instance.
static pt_status validate_batch(const pt_problem* pr, int count, const pt_options* o) {
    if (!pr) return fail(PT_ERR_INVALID, "problems must not be NULL");
    if (!is_pow2(count) || count > 1024) return fail(PT_ERR_INVALID, "count must be a power of two in [1, 1024]");
    for (int b = 0; b < count; ++b) {
        pt_status s = validate(&pr[b], o);
        if (s != PT_OK) return fail(s, "instance " + std::to_string(b) + ": " + g_last_error);
    }
    if (count == 1) return PT_OK;
    const pt_problem& a = pr[0];
    auto same_rect = [](const pt_rect& x, const pt_rect& y) {
        return x.x0 == y.x0 && x.y0 == y.y0 && x.x1 == y.x1 && x.y1 == y.y1;
    };
    for (int b = 1; b < count; ++b) {
        const pt_problem& q = pr[b];
        if (q.n != a.n || q.N != a.N || q.T != a.T)
            return fail(PT_ERR_INVALID, "batch instances must share n, N and T");
        if (q.sigma_in != a.sigma_in || !same_rect(q.sigma_rect, a.sigma_rect) || q.nu_max != a.nu_max)
            return fail(PT_ERR_INVALID, "batch instances must share sigma_in, sigma_rect and nu_max");
    }
    if (o->adjoint) return fail(PT_ERR_INVALID, "adjoint plans take a single problem");
    for (int b = 0; b < count; ++b)
        if (pr[b].nregions > 0) return fail(PT_ERR_INVALID, "region mode takes a single problem");
    if (o->krylov_dim) return fail(PT_ERR_INVALID, "Newton plans take a single problem");
    for (int b = 0; b < count; ++b)
        if (pr[b].d_theta || pr[b].d_sigma || pr[b].d_load)
            return fail(PT_ERR_INVALID, "d_theta, d_sigma and d_load must be NULL in a batch of more than one");
    if ((long)count * (a.N / 2) > 65536) return fail(PT_ERR_INVALID, "count * N / 2 must not exceed 65536");
    return PT_OK;
}

static void layout(Plan& p) {
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t o = off;
        off = align256(off + bytes);
        return o;
    };
    const size_t S = p.ST;  // slots per node over the batch
    const size_t B = p.B;
    p.off_U = take(p.nodes * B * p.N * sizeof(double));
    p.off_F = p.prob.d_load ? take(p.nodes * p.N * sizeof(double)) : 0;
    for (int l = 0; l < p.nlev; ++l) {
        LevelDesc& d = p.lev[l];
        d.off_mt = take(4 * d.nodes * sizeof(double));
        d.off_kt = p.vk ? take(4 * d.nodes * sizeof(double)) : 0;
        d.off_r = take(d.nodes * S * p.elem);
        d.off_x = take(d.nodes * S * p.elem);
    }
    p.off_P = p.lev[0].off_x;
    p.has_cocg_vectors = p.opt.inner == PT_INNER_COCG;
    p.vc_pre = p.opt.vc_cycle == PT_VC_V11 || (p.opt.vc_cycle == PT_VC_DEFAULT && p.opt.inner == PT_INNER_COCG);
    if (p.has_cocg_vectors) {
        size_t v = p.nodes * S * p.elem;
        p.off_cx = take(v);
        p.off_cr = take(v);
        p.off_cq = take(v);
        p.off_cp = take(v);
        // r^H r partials of the vector kernels with their stage-1 tail; five per-slot double2
        // arrays (nr, thr, act, rho, coef) and the active-component counter
        p.off_npart = take((size_t)(cocg_rows(p) + kReduceRows) * S * 3 * sizeof(double));
        p.off_caux = take(5 * S * 2 * sizeof(double) + 16);
    } else {
        p.off_cx = p.off_cr = p.off_cq = p.off_cp = 0;
        p.off_npart = p.off_caux = 0;
    }
    p.off_flags = take(B * 2 * (size_t)p.n * p.n);
    p.off_b = take(B * p.nodes * sizeof(double));
    p.off_rec = take(B * p.nodes * (p.law == PT_NU_EXPCAP ? kRecDoublesExp : kRecDoubles) * sizeof(double));
    p.off_tw64 = take((size_t)p.N * 2 * sizeof(double));
    p.off_tw32 = take((size_t)p.N * 2 * sizeof(float));
    p.off_zs = take(S * 3 * sizeof(double));
    p.off_wave = take(B * (size_t)p.N * sizeof(double));
    p.off_inst = take(B * 4 * sizeof(double));
    p.off_regp = take(B * kMaxRegions * 4 * sizeof(double));
    p.off_rsj = take(kMaxRegions * 2 * sizeof(double));
    p.off_rkh = take(kMaxRegions * sizeof(double));
    // two sets of slot partials (V-cycle and operator sweep), each with its stage-1 tail
    size_t part_slot = (size_t)(p.g_slot0.blocks + kReduceRows + p.g_mv.blocks + kReduceRows) * S * 3;
    size_t part_team = std::max((size_t)p.g_fwd.blocks * p.g_fwd.per_step * 2, (size_t)4096 * 2);
    size_t part_adj = p.opt.adjoint ? std::max<size_t>((size_t)kAdjBlocks * 2, (size_t)p.n * p.n * 2) : 0;
    if (p.opt.krylov_dim > 0) part_adj = std::max<size_t>(part_adj, (size_t)kAdjBlocks * 2);
    p.part_bytes = std::max(std::max(part_slot, part_team), part_adj) * sizeof(double);
    p.off_part = take(p.part_bytes);
    p.off_scal = take(2 * B * sizeof(double));
    p.off_flag = take(sizeof(int));
    if (p.opt.adjoint) {
        p.off_L = take(p.nodes * p.N * sizeof(double));
        p.off_G = take(p.nodes * p.N * sizeof(double));
        p.off_sig = take(2 * (size_t)p.n * p.n * sizeof(double));
    } else {
        p.off_L = p.off_G = p.off_sig = 0;
    }
    if (p.opt.krylov_dim > 0) {
        const size_t tf = p.nodes * p.N * sizeof(double);
        const size_t m = p.opt.krylov_dim;
        p.off_R = take(tf);
        p.off_Ut = take(tf);
        p.off_D = take(tf);
        p.tf_stride = align256(tf);  // byte distance of consecutive basis fields
        p.off_V = take((m + 1) * p.tf_stride);
        p.off_Z = take(m * p.tf_stride);
    } else {
        p.off_R = p.off_Ut = p.off_D = p.off_V = p.off_Z = 0;
        p.tf_stride = 0;
    }
    p.off_coef = take(8 * S * 2 * sizeof(double));  // eight double2 per-slot arrays
    p.off_coef2 = p.off_coef + 4 * S * 2 * sizeof(double);
    p.off_hist = 0;
    p.ws_bytes = off;
}

static void host_tables(Plan& p) {
    const double pi = 3.14159265358979323846;
    p.h_tw64 = new double[2 * p.N];
    p.h_tw32 = new float[2 * p.N];
    for (int k = 0; k < p.N; ++k) {
        double ang = -2.0 * pi * (double)k / (double)p.N;
        p.h_tw64[2 * k] = std::cos(ang);
        p.h_tw64[2 * k + 1] = std::sin(ang);
        p.h_tw32[2 * k] = (float)p.h_tw64[2 * k];
        p.h_tw32[2 * k + 1] = (float)p.h_tw64[2 * k + 1];
    }
    // z_k = (1 - exp(-2 pi i k / N)) / tau: Re = (1 - cos t)/tau, Im = sin t / tau, t = 2 pi k / N
    p.h_zs = new double[3 * (size_t)p.ST];
    for (int s = 0; s < p.S; ++s) {
        double t = 2.0 * pi * (double)s / (double)p.N;
        double re = (1.0 - std::cos(t)) / p.tau, im = std::sin(t) / p.tau;
        if (s == 0) {
            p.h_zs[0] = 0.0;             // k = 0 system on the real part
            p.h_zs[1] = 0.0;
            p.h_zs[2] = 2.0 / p.tau;     // k = N/2 system on the imaginary part
        } else {
            p.h_zs[3 * s] = re;
            p.h_zs[3 * s + 1] = im;
            p.h_zs[3 * s + 2] = re;
        }
    }
    for (int b = 1; b < p.B; ++b) std::memcpy(p.h_zs + 3 * (size_t)b * p.S, p.h_zs, 3 * (size_t)p.S * sizeof(double));
    p.h_wave = new double[(size_t)p.B * p.N];
    p.h_inst = new double[4 * (size_t)p.B];
    for (int b = 0; b < p.B; ++b) {
        const pt_problem& q = p.probs[b];
        for (int j = 0; j < p.N; ++j) {
            double ph = 2.0 * pi * (double)(j + 1) / (double)p.N;  // 2 pi t_{j+1} / T
            p.h_wave[(size_t)b * p.N + j] = (q.waveform == PT_WAVE_SIN) ? std::sin(ph) : std::cos(ph);
        }
        p.h_inst[4 * b] = q.nu_a;
        p.h_inst[4 * b + 1] = q.nu_b;
        p.h_inst[4 * b + 2] = q.nu_out;
        p.h_inst[4 * b + 3] = 0.0;
    }
    // law parameters per region (see law_nu): rectangle problems have region 0 (outside nu_rect:
    // nu_out) and region 1 (inside: nu_a + nu_b s^2/(1+s^2)), both of the rational law
    p.h_regp = new double[(size_t)p.B * kMaxRegions * 4]();
    p.h_rsj = new double[(size_t)kMaxRegions * 2]();
    for (int b = 0; b < p.B; ++b) {
        double* q = p.h_regp + (size_t)b * kMaxRegions * 4;
        if (!p.region_mode) {
            q[0] = p.probs[b].nu_out;
            q[4] = p.probs[b].nu_a;
            q[5] = p.probs[b].nu_b;
            continue;
        }
        for (int r = 0; r < p.nreg; ++r) {
            const pt_region& g = p.regions[r];
            q[4 * r] = g.a;
            q[4 * r + 1] = g.b;
            if (p.law == PT_NU_EXPCAP) {
                q[4 * r + 2] = g.b > 0 ? std::log(g.c) / g.b : 1e300;  // s^2 at which exp(b s^2) = c
                q[4 * r + 3] = g.d;
            }
            p.h_rsj[2 * r] = g.sigma;
            p.h_rsj[2 * r + 1] = g.j;
        }
    }
    for (int r = 0; r < kMaxRegions; ++r)
        p.h_rkh[r] = (p.region_mode && r < p.nreg && p.regions[r].nu_hat > 0) ? p.regions[r].nu_hat : p.prob.nu_max;
}

static pt_status check_ws(const Plan* p, void* ws, size_t bytes) {
    if (!ws) return fail(PT_ERR_WORKSPACE, "workspace is NULL");
    if (((uintptr_t)ws & 255) != 0) return fail(PT_ERR_WORKSPACE, "workspace must be 256-byte aligned");
    if (bytes < p->ws_bytes)
        return fail(PT_ERR_WORKSPACE, "workspace too small: need " + std::to_string(p->ws_bytes) + " bytes");
    return PT_OK;
}

// Per-kernel timing for one pt_solve call: events are created once per plan.
static pt_status timer_start(Plan& p) {
    if (!p.opt.timing) return PT_OK;
    if (!p.tm) {
        p.tm = new (std::nothrow) Timer();
        if (!p.tm) return fail(PT_ERR_INVALID, "out of host memory");
        for (int i = 0; i < 2 * Timer::kCap; ++i) PT_HIP(hipEventCreate(&p.tm->ev[i]));
    }
    p.tm->on = true;
    p.tm->mask = p.opt.timing_mask ? (unsigned)p.opt.timing_mask : ~0u;
    p.tm->used = 0;
    for (int c = 0; c < KID_COUNT; ++c) {
        p.tm->ms[c] = 0.0;
        p.tm->cnt[c] = 0;
    }
    return PT_OK;
}

// Upload the small tables and build the per-level operators in the workspace.
static pt_status setup(Plan& p, char* ws, hipStream_t st) {
    PT_HIP(hipMemcpyAsync(ws + p.off_tw64, p.h_tw64, (size_t)p.N * 2 * sizeof(double), hipMemcpyHostToDevice, st));
    PT_HIP(hipMemcpyAsync(ws + p.off_tw32, p.h_tw32, (size_t)p.N * 2 * sizeof(float), hipMemcpyHostToDevice, st));
    PT_HIP(hipMemcpyAsync(ws + p.off_zs, p.h_zs, (size_t)p.ST * 3 * sizeof(double), hipMemcpyHostToDevice, st));
    PT_HIP(hipMemcpyAsync(ws + p.off_wave, p.h_wave, (size_t)p.B * p.N * sizeof(double), hipMemcpyHostToDevice, st));
    PT_HIP(hipMemcpyAsync(ws + p.off_inst, p.h_inst, (size_t)p.B * 4 * sizeof(double), hipMemcpyHostToDevice, st));
    PT_HIP(hipMemcpyAsync(ws + p.off_regp, p.h_regp, (size_t)p.B * kMaxRegions * 4 * sizeof(double),
                          hipMemcpyHostToDevice, st));
    PT_HIP(hipMemcpyAsync(ws + p.off_rsj, p.h_rsj, (size_t)kMaxRegions * 2 * sizeof(double), hipMemcpyHostToDevice, st));
    PT_HIP(hipMemcpyAsync(ws + p.off_rkh, p.h_rkh, (size_t)kMaxRegions * sizeof(double), hipMemcpyHostToDevice, st));
    TM(KID_SETUP, launch_setup_fine(p, ws, st));
    for (int l = 0; l + 1 < p.nlev; ++l) TM(KID_SETUP, launch_galerkin(p, ws, l, st));
    if (p.vk) {
        // Khat = S_nuhat on the finest level and its Galerkin coarsening (same stencil layout)
        TM(KID_SETUP, launch_setup_stiffness(p, ws, st));
        for (int l = 0; l + 1 < p.nlev; ++l) TM(KID_SETUP, launch_galerkin_table(p, ws, l, true, st));
    }
    TM(KID_SETUP, launch_row_records(p, ws, st));
    PT_HIP(hipGetLastError());
    return PT_OK;
}

// Approximate X = (Khat + z M)^{-1} Rhat for every slot. On return *X and *coef describe
// the correction coef (x) X (coef NULL means identity).
static pt_status inner_solve(Plan& p, char* ws, hipStream_t st, int iters, const void** X, const double** coef,
                             bool capture = false) {
    double* part = (double*)(ws + p.off_part);
    double2* cf = (double2*)(ws + p.off_coef);
    const size_t S = p.ST;
    double* num = (double*)(cf + 0 * S);
    double* den = (double*)(cf + 1 * S);
    double* alpha = (double*)(cf + 2 * S);
    int* flag = (int*)(ws + p.off_flag);
    void* R = ws + p.lev[0].off_r;
    void* P = ws + p.off_P;
    if (p.opt.inner == PT_INNER_GALERKIN1) {
        // p^H r partials from the V-cycle's last sweep, p^H A p partials after them; both reduced
        // and divided in two launches
        double* part_b = part + (size_t)(p.g_slot0.blocks + kReduceRows) * S * 3;
        launch_vcycle(p, ws, R, P, DOT_HERM, part, st);
        TM(KID_MATVEC, launch_matvec(p, ws, P, nullptr, DOT_HERM, part_b, st));
        TM(KID_REDUCE, launch_reduce_ratio(p, part, p.g_slot0.blocks, part_b, p.g_mv.blocks, DOT_HERM, num, den, alpha,
                                           st));
        p.inner_done = 1;
        *X = P;
        *coef = alpha;
        return PT_OK;
    }
    // COCG from zero (x = 0, r = Rhat, z = B r, p = z, rho = r^T z), per frequency until
    // ||r_k|| <= inner_rtol ||Rhat_k|| (then masked: alpha = beta = 0, so x_k and r_k stay as
    // they are) or `iters` steps. Slot 0's two real systems are tested and masked apart.
    void* x = ws + p.off_cx;
    void* r = ws + p.off_cr;
    void* q = ws + p.off_cq;
    void* pv = ws + p.off_cp;
    void* z = P;
    double* npart = (double*)(ws + p.off_npart);
    double2* aux = (double2*)(ws + p.off_caux);
    CocgScalars cs;
    cs.nr = (double*)(aux + 0 * S);
    cs.thr = (double*)(aux + 1 * S);
    cs.act = (double*)(aux + 2 * S);
    cs.rho = (double*)(aux + 3 * S);
    cs.coef = (double*)(aux + 4 * S);
    cs.count = (int*)(aux + 5 * S);
    cs.flag = flag;
    cs.eta2 = p.opt.inner_rtol * p.opt.inner_rtol;
    cs.btol = p.opt.breakdown_tol > 0 ? p.opt.breakdown_tol : (p.fp32 ? 64.0 * 5.96e-8 : 64.0 * 1.11e-16);
    const int nrows = cocg_rows(p);
    const bool early = p.opt.inner_rtol > 0 && !capture;  // host test between steps (not in a graph)
    TM(KID_MEMSET, launch_zero16(x, p.nodes * S * p.elem, st));
    TM(KID_COCG, launch_cocg_vec(p, 1, nullptr, nullptr, r, R, nullptr, npart, st));
    TM(KID_REDUCE, launch_cocg_reduce(p, npart, nrows, COCG_NORM0, cs, st));
    launch_vcycle(p, ws, r, z, DOT_BILIN, part, st);
    TM(KID_REDUCE, launch_cocg_reduce(p, part, p.g_slot0.blocks, COCG_RHO, cs, st));
    TM(KID_COCG, launch_copy_slots(p, z, pv, st));
    int done = 0;
    for (int it = 0; it < iters; ++it) {
        TM(KID_MATVEC, launch_matvec(p, ws, pv, q, DOT_BILIN, part, st));
        TM(KID_REDUCE, launch_cocg_reduce(p, part, p.g_mv.blocks, COCG_ALPHA, cs, st));
        TM(KID_COCG, launch_cocg_vec(p, 0, cs.coef, x, r, pv, q, npart, st));
        TM(KID_MEMSET, launch_zero16(cs.count, 16, st));
        TM(KID_REDUCE, launch_cocg_reduce(p, npart, nrows, COCG_NORM, cs, st));
        done = it + 1;
        if (early) {
            int active = 0;
            PT_HIP(hipMemcpyAsync(&active, cs.count, sizeof(int), hipMemcpyDeviceToHost, st));
            PT_HIP(hipStreamSynchronize(st));
            if (active == 0) break;
        }
        if (it + 1 == iters) break;
        launch_vcycle(p, ws, r, z, DOT_BILIN, part, st);
        TM(KID_REDUCE, launch_cocg_reduce(p, part, p.g_slot0.blocks, COCG_BETA, cs, st));
        TM(KID_COCG, launch_cocg_p(p, cs.coef, z, pv, st));
    }
    p.inner_done = done;
    *X = x;
    *coef = nullptr;
    PT_HIP(hipGetLastError());
    return PT_OK;
}

// ---------------------------------------------------------------- outer loop

// Graph of check_every outer steps, captured once per plan and workspace.
struct GraphCache {
    hipStream_t cap = nullptr;  // capture stream (default priority)
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    char* ws = nullptr;  // workspace the graph's kernel arguments point into
    int steps = 0;
    bool adjoint = false;
    long long inner_per_launch = 0;  // inner steps of the captured segment
    int inner_max = 0;
};

void graph_release(Plan& p) {
    GraphCache* g = p.gr;
    if (!g) return;
    if (g->exec) hipGraphExecDestroy(g->exec);
    if (g->graph) hipGraphDestroy(g->graph);
    if (g->cap) hipStreamDestroy(g->cap);
    delete g;
    p.gr = nullptr;
}

// Residual of the current iterate into Rhat (frequency domain, solver precision) and its
// norm partials reduced into scal. Forward: R = F - A(U). Adjoint: R = dl/dU - J^T lambda,
// transformed with conjugated shifts (the DFT of the backward-in-time coupling).
static void residual_step(Plan& p, char* ws, bool adjoint, hipStream_t st) {
    double* part = (double*)(ws + p.off_part);
    double* scal = (double*)(ws + p.off_scal);
    if (!adjoint) {
        const int flat = launch_forward(p, ws, TM_RESIDUAL, (double*)(ws + p.off_U), ws + p.lev[0].off_r, nullptr,
                                        part, st);
        TM(KID_REDUCE, launch_reduce_norms(p, ws, part, flat, scal, st));
        return;
    }
    int nparts = 0;
    TM(KID_RESIDUAL, nparts = launch_adj_residual(p, ws, ws + p.off_P, st));
    TM(KID_REDUCE, launch_reduce_pairs(p, part, nparts, scal, st));
    launch_rfft(p, ws, ws + p.off_P, ws + p.lev[0].off_r, 1, st);
}

// One fixed-point update once the residual of the iterate is in Rhat (eq. (iter2) in
// correction form, U^{k+1} = U^k + P^{-1} R^k; for the adjoint with the transposed P),
// followed by the residual of the new iterate and its norm partials.
static pt_status outer_segment(Plan& p, char* ws, bool adjoint, hipStream_t st, bool capture = false) {
    double* X0 = (double*)(ws + (adjoint ? p.off_L : p.off_U));
    const void* X = nullptr;
    const double* coef = nullptr;
    pt_status s = inner_solve(p, ws, st, p.opt.inner_iters, &X, &coef, capture);
    if (s != PT_OK) return s;
    p.inner_max = std::max(p.inner_max, p.inner_done);
    p.inner_sum += p.inner_done;
    TM(KID_INVERSE, launch_inverse(p, ws, X, coef, X0, 1, st, adjoint ? 1 : 0));
    residual_step(p, ws, adjoint, st);
    return PT_OK;
}

static pt_status graph_get(Plan& p, char* ws, int steps, bool adjoint, hipGraphExec_t* exec) {
    if (!p.gr) {
        p.gr = new (std::nothrow) GraphCache();
        if (!p.gr) return fail(PT_ERR_INVALID, "out of host memory");
        PT_HIP(hipStreamCreateWithFlags(&p.gr->cap, hipStreamNonBlocking));
    }
    GraphCache* g = p.gr;
    if (g->exec && g->ws == ws && g->steps == steps && g->adjoint == adjoint) {
        *exec = g->exec;
        return PT_OK;
    }
    if (g->exec) hipGraphExecDestroy(g->exec);
    if (g->graph) hipGraphDestroy(g->graph);
    g->exec = nullptr;
    g->graph = nullptr;
    PT_HIP(hipStreamBeginCapture(g->cap, hipStreamCaptureModeThreadLocal));
    pt_status s = PT_OK;
    // the capture only records the launches: the inner-step counters are restored and every
    // replay adds the captured segment's steps
    const long long sum0 = p.inner_sum;
    const int max0 = p.inner_max;
    p.inner_max = 0;
    for (int i = 0; i < steps && s == PT_OK; ++i) s = outer_segment(p, ws, adjoint, g->cap, true);
    g->inner_per_launch = p.inner_sum - sum0;
    g->inner_max = p.inner_max;
    p.inner_sum = sum0;
    p.inner_max = max0;
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(g->cap, &graph);
    if (s != PT_OK) {
        if (graph) hipGraphDestroy(graph);
        return s;
    }
    if (e != hipSuccess) return fail(PT_ERR_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
    e = hipGraphInstantiate(&g->exec, graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        hipGraphDestroy(graph);
        return fail(PT_ERR_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
    }
    g->graph = graph;
    g->ws = ws;
    g->steps = steps;
    g->adjoint = adjoint;
    *exec = g->exec;
    return PT_OK;
}

struct EventPair {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~EventPair() {
        if (e0) hipEventDestroy(e0);
        if (e1) hipEventDestroy(e1);
    }
};

// The fixed-point iteration (eqs. (iter1)-(iter2)) for the B instances of a plan, stopped
// when every instance's relative residual is at most tol. d_u: [B][N][n+1][n+1];
// stats: NULL or an array of B. Adjoint (B = 1): the same iteration for J^T lambda = dl/dU
// at the state d_u, lambda in and out through d_lambda.
// no_alloc: create no HIP object (events), time the call on the host clock (it blocks anyway).
static pt_status solve_impl(Plan& p, void* d_ws, size_t ws_bytes, double* d_u, hipStream_t st, pt_stats* stats,
                            bool adjoint = false, double* d_lambda = nullptr, bool no_alloc = false) {
    pt_status s = check_ws(&p, d_ws, ws_bytes);
    if (s != PT_OK) return s;
    char* ws = (char*)d_ws;
    const int B = p.B;
    EventPair ev;
    const auto host_t0 = std::chrono::steady_clock::now();
    if (!no_alloc) {
        PT_HIP(hipEventCreate(&ev.e0));
        PT_HIP(hipEventCreate(&ev.e1));
    }
    s = timer_start(p);
    if (s != PT_OK) return s;
    p.inner_max = 0;
    p.inner_sum = 0;
    if (!no_alloc) PT_HIP(hipEventRecord(ev.e0, st));
    s = setup(p, ws, st);
    if (s != PT_OK) return s;
    double* U = (double*)(ws + p.off_U);
    double* X0 = adjoint ? (double*)(ws + p.off_L) : U;   // the iterate
    double* d_x = adjoint ? d_lambda : d_u;
    if (p.prob.d_load) TM(KID_TRANSPOSE, launch_transpose_in(p, p.prob.d_load, (double*)(ws + p.off_F), st));
    if (adjoint) TM(KID_TRANSPOSE, launch_transpose_in(p, d_u, U, st));
    if (p.opt.use_initial_guess)
        TM(KID_TRANSPOSE, launch_transpose_in(p, d_x, X0, st));
    else
        TM(KID_MEMSET, launch_zero16(X0, (size_t)B * p.nodes * p.N * sizeof(double), st));
    if (adjoint) TM(KID_OTHER, launch_adj_source(p, ws, st));
    double* scal = (double*)(ws + p.off_scal);
    int* flag = (int*)(ws + p.off_flag);
    TM(KID_MEMSET, launch_zero16(flag, 16, st));
    std::vector<double> h(2 * (size_t)B), rel(B, INFINITY), fnorm(B, 0.0), best(B, INFINITY), d0(B, 0.0);
    std::vector<int> conv(B, -1);
    const int ce = p.opt.check_every;
    int hist = 0;
    // One run of the iteration from the current iterate (whose residual step has been
    // launched) until every instance meets tol, a failure, or max_steps updates. relative0:
    // divide by the residual of the starting iterate instead of ||F||.
    auto run = [&](double tol, int max_steps, bool record, bool relative0, int& k, pt_status& result) -> pt_status {
        std::fill(best.begin(), best.end(), INFINITY);
        std::fill(conv.begin(), conv.end(), -1);
        result = PT_ERR_NOT_CONVERGED;
        k = 0;
        for (;;) {
            bool last = (k >= max_steps);
            if (last || k % ce == 0) {
                int hflag = 0;
                PT_HIP(hipMemcpyAsync(h.data(), scal, 2 * (size_t)B * sizeof(double), hipMemcpyDeviceToHost, st));
                PT_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
                PT_HIP(hipStreamSynchronize(st));
                PT_HIP(hipGetLastError());
                tm_flush(p);
                bool all = true;
                int bad = -1;
                for (int b = 0; b < B; ++b) {
                    const double r2 = h[2 * b], f2 = h[2 * b + 1];
                    fnorm[b] = std::sqrt(f2);
                    if (k == 0) d0[b] = std::sqrt(r2);
                    if (relative0)
                        rel[b] = d0[b] > 0 ? std::sqrt(r2) / d0[b] : 0.0;
                    else
                        rel[b] = (f2 > 0) ? std::sqrt(r2 / f2) : std::sqrt(r2);
                    if (record && stats && stats[b].residual_history && hist < stats[b].history_cap)
                        stats[b].residual_history[hist] = rel[b];
                    if (!std::isfinite(rel[b]) && bad < 0) bad = b;
                    if (rel[b] <= tol) {
                        if (conv[b] < 0) conv[b] = k;
                    } else {
                        all = false;
                    }
                }
                if (record) ++hist;
                if (log_level() >= 2)
                    for (int b = 0; b < B; ++b)
                        PT_LOG(2, "%s step %d%s: rel %.6e", adjoint ? "adjoint" : "outer", k,
                               B > 1 ? (" instance " + std::to_string(b)).c_str() : "", rel[b]);
                auto inst = [&](int b) { return B > 1 ? " (instance " + std::to_string(b) + ")" : std::string(); };
                if (bad >= 0) {
                    result = fail(PT_ERR_NONFINITE,
                                  "residual norm is not finite at outer step " + std::to_string(k) + inst(bad));
                    return PT_OK;
                }
                if (hflag) {
                    result = fail(PT_ERR_BREAKDOWN, "COCG breakdown before outer step " + std::to_string(k));
                    return PT_OK;
                }
                if (all) {
                    result = PT_OK;
                    return PT_OK;
                }
                int grew = -1;
                for (int b = 0; b < B; ++b) {
                    if (rel[b] < best[b]) best[b] = rel[b];
                    if (grew < 0 && p.opt.diverge_factor > 0 && rel[b] > p.opt.diverge_factor * best[b]) grew = b;
                }
                if (grew >= 0) {
                    result = fail(PT_ERR_DIVERGED, "residual grew by more than diverge_factor at outer step " +
                                                       std::to_string(k) + inst(grew));
                    return PT_OK;
                }
            }
            if (last) {
                result = fail(PT_ERR_NOT_CONVERGED, "max_outer reached");
                return PT_OK;
            }
            if (p.opt.graph && k % ce == 0 && k + ce <= max_steps) {
                hipGraphExec_t exec = nullptr;
                pt_status g = graph_get(p, ws, ce, adjoint, &exec);
                if (g != PT_OK) return g;
                PT_HIP(hipGraphLaunch(exec, st));
                p.inner_sum += p.gr->inner_per_launch;
                p.inner_max = std::max(p.inner_max, p.gr->inner_max);
                k += ce;
            } else {
                pt_status g = outer_segment(p, ws, adjoint, st);
                if (g != PT_OK) return g;
                ++k;
            }
        }
    };
    pt_status result = PT_OK;
    int k = 0, init_iters = 0;
    if (p.opt.init_static && !adjoint) {
        // Static start (Sec. 4, "Initialization"): the decoupled problems K(u^n) = f^n of sigma = 0,
        // i.e. the same iteration with every mass table zeroed; then the tables are rebuilt.
        for (int l = 0; l < p.nlev; ++l) TM(KID_MEMSET, launch_zero16(ws + p.lev[l].off_mt, 4 * p.lev[l].nodes * sizeof(double), st));
        TM(KID_SETUP, launch_row_records(p, ws, st));
        residual_step(p, ws, false, st);
        s = run(p.opt.init_tol, p.opt.max_outer, false, false, init_iters, result);
        if (s != PT_OK) return s;
        if (result == PT_ERR_NOT_CONVERGED) result = PT_OK;  // the start need not be exact
        TM(KID_SETUP, launch_setup_fine(p, ws, st));
        for (int l = 0; l + 1 < p.nlev; ++l) TM(KID_SETUP, launch_galerkin(p, ws, l, st));
        TM(KID_SETUP, launch_row_records(p, ws, st));
    }
    if (result == PT_OK) {
        residual_step(p, ws, adjoint, st);
        s = run(p.opt.tol, p.opt.max_outer, true, p.opt.stop_relative_initial != 0, k, result);
        if (s != PT_OK) return s;
    }
    TM(KID_TRANSPOSE, launch_transpose_out(p, X0, d_x, st));
    float ms = 0.f;
    if (no_alloc) {
        PT_HIP(hipStreamSynchronize(st));
        PT_HIP(hipGetLastError());
        ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - host_t0).count();
    } else {
        PT_HIP(hipEventRecord(ev.e1, st));
        PT_HIP(hipEventSynchronize(ev.e1));
        PT_HIP(hipGetLastError());
        PT_HIP(hipEventElapsedTime(&ms, ev.e0, ev.e1));
    }
    tm_flush(p);
    PT_LOG(1, "%s n=%d N=%d B=%d %s: %s after %d steps (static start %d), rel %.3e, inner steps %lld (max %d), %.2f ms",
           adjoint ? "adjoint" : "solve", p.n, p.N, B, p.fp32 ? "fp32+refine" : "fp64", pt_status_string(result), k,
           init_iters, *std::max_element(rel.begin(), rel.end()), p.inner_sum, p.inner_max, ms);
    if (stats) {
        for (int b = 0; b < B; ++b) {
            pt_stats& o = stats[b];
            o.outer_iters = k;
            o.rel_residual = rel[b];
            o.f_norm = fnorm[b];
            o.time_ms = ms;
            o.history_len = hist < o.history_cap ? hist : o.history_cap;
            o.converged_at = conv[b];
            o.init_iters = init_iters;
            o.rel_initial = fnorm[b] > 0 ? d0[b] / fnorm[b] : d0[b];
            o.inner_iters_max = p.inner_max;
            o.inner_iters_sum = p.inner_sum;
            for (int c = 0; c < KID_COUNT; ++c) {
                if (o.kernel_ms) o.kernel_ms[c] = p.tm ? p.tm->ms[c] : 0.0;
                if (o.kernel_launches) o.kernel_launches[c] = p.tm ? p.tm->cnt[c] : 0;
            }
        }
    }
    if (p.tm) p.tm->on = false;
    return result;
}

// ---------------------------------------------------------------- Newton outer loop

// Newton's method on A(U) = F with flexible GMRES for the steps and Armijo backtracking
// (method (M2) of Sec. 4 with the periodic solve of the fixed-point iteration in place of
// multigrid in time as the preconditioner).
static pt_status newton_impl(Plan& p, void* d_ws, size_t ws_bytes, double* d_u, hipStream_t st, pt_stats* stats) {
    pt_status s = check_ws(&p, d_ws, ws_bytes);
    if (s != PT_OK) return s;
    char* ws = (char*)d_ws;
    EventPair ev;
    PT_HIP(hipEventCreate(&ev.e0));
    PT_HIP(hipEventCreate(&ev.e1));
    s = timer_start(p);
    if (s != PT_OK) return s;
    p.inner_max = 0;
    p.inner_sum = 0;
    PT_HIP(hipEventRecord(ev.e0, st));
    s = setup(p, ws, st);
    if (s != PT_OK) return s;
    const int m = p.opt.krylov_dim;
    double* U = (double*)(ws + p.off_U);
    double* R = (double*)(ws + p.off_R);
    double* Ut = (double*)(ws + p.off_Ut);
    double* D = (double*)(ws + p.off_D);
    auto Vf = [&](int i) { return (double*)(ws + p.off_V + (size_t)i * p.tf_stride); };
    auto Zf = [&](int i) { return (double*)(ws + p.off_Z + (size_t)i * p.tf_stride); };
    double* part = (double*)(ws + p.off_part);
    double* scal = (double*)(ws + p.off_scal);
    if (p.prob.d_load) launch_transpose_in(p, p.prob.d_load, (double*)(ws + p.off_F), st);
    if (p.opt.use_initial_guess)
        launch_transpose_in(p, d_u, U, st);
    else
        launch_zero16(U, p.nodes * p.N * sizeof(double), st);
    double h2[2];
    auto fetch2 = [&]() -> pt_status {
        PT_HIP(hipMemcpyAsync(h2, scal, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
        PT_HIP(hipStreamSynchronize(st));
        PT_HIP(hipGetLastError());
        return PT_OK;
    };
    // ||F - A(X)|| and ||F|| with the residual (FP64, node-major) into Rout
    auto residual = [&](const double* X, double* Rout, double& r, double& f) -> pt_status {
        const int flat = launch_forward(p, ws, TM_RESIDUAL, X, nullptr, Rout, part, st);
        launch_reduce_norms(p, ws, part, flat, scal, st);
        pt_status q = fetch2();
        r = std::sqrt(h2[0]);
        f = std::sqrt(h2[1]);
        return q;
    };
    auto dot = [&](const double* a, const double* b, double& out) -> pt_status {
        const int np = launch_tdot(p, a, b, part, st);
        launch_reduce_pairs(p, part, np, scal, st);
        pt_status q = fetch2();
        out = h2[0];
        return q;
    };
    // z = P^{-1} v: time DFT, the inner method per frequency, inverse DFT
    auto precond = [&](const double* v, double* z) -> pt_status {
        launch_forward(p, ws, TM_SIGNAL, v, ws + p.lev[0].off_r, nullptr, part, st);
        const void* X = nullptr;
        const double* coef = nullptr;
        pt_status q = inner_solve(p, ws, st, p.opt.inner_iters, &X, &coef);
        if (q != PT_OK) return q;
        p.inner_max = std::max(p.inner_max, p.inner_done);
        p.inner_sum += p.inner_done;
        launch_inverse(p, ws, X, coef, z, 0, st);
        return PT_OK;
    };
    double r = 0, f = 0, d0 = 0, rel = INFINITY;
    s = residual(U, R, r, f);
    if (s != PT_OK) return s;
    d0 = r;
    pt_status result = PT_ERR_NOT_CONVERGED;
    int k = 0, hist = 0, kry = 0;
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m);
    auto Hc = [&](int i, int j) -> double& { return H[(size_t)i * m + j]; };
    for (;;) {
        const double den = p.opt.stop_relative_initial ? d0 : f;
        rel = den > 0 ? r / den : r;
        if (stats && stats->residual_history && hist < stats->history_cap) stats->residual_history[hist] = rel;
        ++hist;
        if (!std::isfinite(rel)) {
            result = fail(PT_ERR_NONFINITE, "residual norm is not finite at Newton step " + std::to_string(k));
            break;
        }
        if (rel <= p.opt.tol) {
            result = PT_OK;
            break;
        }
        if (k >= p.opt.max_outer) {
            result = fail(PT_ERR_NOT_CONVERGED, "max_outer reached");
            break;
        }
        // flexible GMRES for J D = R from D = 0
        launch_zero16(D, p.nodes * p.N * sizeof(double), st);
        double beta = r;
        launch_taxpby(p, 1.0 / beta, R, 0.0, Vf(0), st);
        int steps_here = 0;
        for (;;) {
            std::fill(g.begin(), g.end(), 0.0);
            g[0] = beta;
            int jd = 0;
            double est = beta;
            for (int j = 0; j < m; ++j) {
                s = precond(Vf(j), Zf(j));
                if (s != PT_OK) return s;
                launch_jac_apply(p, ws, Zf(j), nullptr, Vf(j + 1), +1, st);
                for (int i = 0; i <= j; ++i) {  // modified Gram-Schmidt
                    double hij = 0;
                    s = dot(Vf(j + 1), Vf(i), hij);
                    if (s != PT_OK) return s;
                    Hc(i, j) = hij;
                    launch_taxpby(p, -hij, Vf(i), 1.0, Vf(j + 1), st);
                }
                double nn = 0;
                s = dot(Vf(j + 1), Vf(j + 1), nn);
                if (s != PT_OK) return s;
                const double hn = std::sqrt(nn);
                Hc(j + 1, j) = hn;
                if (hn > 0) launch_taxpby(p, 1.0 / hn, Vf(j + 1), 0.0, Vf(j + 1), st);
                for (int i = 0; i < j; ++i) {  // previous Givens rotations on column j
                    const double a0 = Hc(i, j), a1 = Hc(i + 1, j);
                    Hc(i, j) = cs[i] * a0 + sn[i] * a1;
                    Hc(i + 1, j) = -sn[i] * a0 + cs[i] * a1;
                }
                const double a0 = Hc(j, j), a1 = Hc(j + 1, j), rr = std::hypot(a0, a1);
                cs[j] = rr > 0 ? a0 / rr : 1.0;
                sn[j] = rr > 0 ? a1 / rr : 0.0;
                Hc(j, j) = rr;
                Hc(j + 1, j) = 0.0;
                g[j + 1] = -sn[j] * g[j];
                g[j] = cs[j] * g[j];
                est = std::fabs(g[j + 1]);
                jd = j + 1;
                ++steps_here;
                ++kry;
                if (est <= p.opt.forcing * r || hn == 0.0 || steps_here >= p.opt.max_krylov) break;
            }
            for (int i = jd - 1; i >= 0; --i) {  // H y = g, upper triangular
                double sacc = g[i];
                for (int l = i + 1; l < jd; ++l) sacc -= Hc(i, l) * y[l];
                y[i] = Hc(i, i) != 0.0 ? sacc / Hc(i, i) : 0.0;
            }
            for (int i = 0; i < jd; ++i) launch_taxpby(p, y[i], Zf(i), 1.0, D, st);
            if (est <= p.opt.forcing * r || steps_here >= p.opt.max_krylov) break;
            // restart from the true residual R - J D
            launch_jac_apply(p, ws, D, R, Vf(0), +1, st);
            double bb = 0;
            s = dot(Vf(0), Vf(0), bb);
            if (s != PT_OK) return s;
            beta = std::sqrt(bb);
            if (!(beta > 0)) break;
            launch_taxpby(p, 1.0 / beta, Vf(0), 0.0, Vf(0), st);
        }
        // Armijo backtracking on ||F - A(U + lambda D)||
        double lam = 1.0;
        bool accepted = false;
        double* Rt = Vf(0);
        for (int ls = 0; ls < 30; ++ls) {
            launch_taxpby(p, 1.0, U, 0.0, Ut, st);
            launch_taxpby(p, lam, D, 1.0, Ut, st);
            double rt = 0, ft = 0;
            s = residual(Ut, Rt, rt, ft);
            if (s != PT_OK) return s;
            if (std::isfinite(rt) && rt <= (1.0 - 1e-4 * lam) * r) {
                launch_taxpby(p, 1.0, Ut, 0.0, U, st);
                launch_taxpby(p, 1.0, Rt, 0.0, R, st);
                r = rt;
                accepted = true;
                break;
            }
            lam *= 0.5;
        }
        if (!accepted) {
            result = fail(PT_ERR_NOT_CONVERGED, "line search failed at Newton step " + std::to_string(k));
            break;
        }
        ++k;
    }
    launch_transpose_out(p, U, d_u, st);
    PT_HIP(hipEventRecord(ev.e1, st));
    PT_HIP(hipEventSynchronize(ev.e1));
    PT_HIP(hipGetLastError());
    tm_flush(p);
    float ms = 0.f;
    PT_HIP(hipEventElapsedTime(&ms, ev.e0, ev.e1));
    if (stats) {
        stats->outer_iters = k;
        stats->rel_residual = rel;
        stats->f_norm = f;
        stats->time_ms = ms;
        stats->history_len = hist < stats->history_cap ? hist : stats->history_cap;
        stats->converged_at = result == PT_OK ? k : -1;
        stats->init_iters = 0;
        stats->rel_initial = f > 0 ? d0 / f : d0;
        stats->krylov_iters = kry;
        stats->inner_iters_max = p.inner_max;
        stats->inner_iters_sum = p.inner_sum;
        for (int c = 0; c < KID_COUNT; ++c) {
            if (stats->kernel_ms) stats->kernel_ms[c] = p.tm ? p.tm->ms[c] : 0.0;
            if (stats->kernel_launches) stats->kernel_launches[c] = p.tm ? p.tm->cnt[c] : 0;
        }
    }
    if (p.tm) p.tm->on = false;
    return result;
}

pt_status check_bounds(const Plan& p, std::string& msg);

// ---------------------------------------------------------------- allocation-free solve

// Device scratch of pt_solve_noalloc: the solver's whole workspace lives here. Every GPU the
// library runs on holds its own copy until the process ends. In host code the name only
// stands for the symbol: kernels and copies get the device address that hipGetSymbolAddress
// returns for the current device (scratch_address).
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static void* g_scratch_ptr[kMaxDevices];

// Device address of scratch on the current device, looked up once per device (with that
// device current) and kept.
static pt_status scratch_address(void** out) {
    int dev = -1;
    PT_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(PT_ERR_INVALID, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess)
            return fail(PT_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        if (!ptr || ((uintptr_t)ptr & 255) != 0)
            return fail(PT_ERR_HIP, "scratch has no 256-byte aligned device address");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return PT_OK;
}

}  // namespace pt

using namespace pt;

struct pt_plan {
    Plan p;
};

extern "C" {

int32_t pt_version(void) { return 1; }

const char* pt_last_error(void) { return g_last_error.c_str(); }

const char* pt_kernel_class_name(int32_t id) {
    static const char* names[KID_COUNT] = {"setup",   "transpose", "residual_sweep", "rfft", "reductions",
                                           "vcycle_down_fine", "vcycle_down_coarse", "vcycle_coarsest",
                                           "vcycle_up_fine",   "vcycle_up_coarse",   "matvec_dot",
                                           "inverse_rfft_update", "cocg_update", "memset", "other"};
    if (id < 0 || id >= KID_COUNT) return nullptr;
    return names[id];
}

const char* pt_status_string(pt_status s) {
    switch (s) {
        case PT_OK: return "PT_OK";
        case PT_ERR_INVALID: return "PT_ERR_INVALID";
        case PT_ERR_HIP: return "PT_ERR_HIP";
        case PT_ERR_NOT_CONVERGED: return "PT_ERR_NOT_CONVERGED";
        case PT_ERR_BREAKDOWN: return "PT_ERR_BREAKDOWN";
        case PT_ERR_NONFINITE: return "PT_ERR_NONFINITE";
        case PT_ERR_DIVERGED: return "PT_ERR_DIVERGED";
        case PT_ERR_WORKSPACE: return "PT_ERR_WORKSPACE";
    }
    return "PT_UNKNOWN_STATUS";
}

void pt_options_default(pt_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-8;
    o->max_outer = 1000;
    o->check_every = 1;
    o->precision = PT_FP64;
    o->inner = PT_INNER_GALERKIN1;
    o->inner_iters = 1;
    o->vc_sweeps = 1;
    o->vc_omega = 0.8;
    o->use_initial_guess = 0;
    o->diverge_factor = 1e3;
    o->xcd_remap = 1;
    o->init_tol = 1e-8;
    o->forcing = 1e-2;
    o->max_krylov = 100;
}

static pt_status plan_create_impl(const pt_problem* probs, int count, const pt_options* opts, pt_plan** out) {
    if (!out) return fail(PT_ERR_INVALID, "out must not be NULL");
    *out = nullptr;
    pt_status s = validate_batch(probs, count, opts);
    if (s != PT_OK) return s;
    if (opts->graph && opts->timing)
        return fail(PT_ERR_INVALID, "graph replay and per-kernel timing cannot be combined");
    pt_plan* h = new (std::nothrow) pt_plan();
    if (!h) return fail(PT_ERR_INVALID, "out of host memory");
    Plan& p = h->p;
    const pt_problem* prob = &probs[0];
    p.prob = *prob;
    p.opt = *opts;
    p.B = count;
    p.probs = new pt_problem[count];
    for (int b = 0; b < count; ++b) p.probs[b] = probs[b];
    p.law = prob->law;
    p.region_mode = prob->nregions > 0;
    p.nreg = p.region_mode ? prob->nregions : 2;
    if (p.region_mode) std::copy(prob->regions, prob->regions + prob->nregions, p.regions);
    p.vk = false;
    for (int r = 0; p.region_mode && r < p.nreg; ++r) p.vk = p.vk || p.regions[r].nu_hat > 0;
    p.prob.regions = nullptr;  // the caller's array need not outlive the plan
    for (int b = 0; b < count; ++b) p.probs[b].regions = nullptr;
    p.n = prob->n;
    p.N = prob->N;
    p.S = prob->N / 2;
    p.ST = p.B * p.S;
    p.side = p.n + 1;
    p.nodes = (size_t)p.side * p.side;
    p.fp32 = opts->precision == PT_FP32_REFINE;
    p.elem = p.fp32 ? 2 * sizeof(float) : 2 * sizeof(double);
    p.tau = prob->T / prob->N;
    p.h = 1.0 / prob->n;
    p.nlev = 0;
    for (int nn = p.n; nn >= 2; nn /= 2) {
        LevelDesc& d = p.lev[p.nlev++];
        d.n = nn;
        d.side = nn + 1;
        d.nodes = (size_t)d.side * d.side;
    }
    p.tm = nullptr;
    p.gr = nullptr;
    p.target_slot = opts->grid_slot > 0 ? opts->grid_slot : 8192;
    p.target_team = opts->grid_team > 0 ? opts->grid_team : 262144;
    p.target_down = opts->grid_restrict > 0 ? opts->grid_restrict : p.target_slot;
    p.target_up = opts->grid_up > 0 ? opts->grid_up : p.target_slot;
    p.g_slot0 = slot_geom(p.side, p.ST, p.fp32 ? 2 : 1, p.target_up);
    // operator sweep: 64-lane slot chunks, so a workgroup holds four column pairs and their
    // shared halo columns come through L1 (1024^2 x 512: 0.508 -> 0.490 ms FP32, 0.930 -> 0.891 ms FP64)
    p.g_mv = slot_geom(p.side, p.ST, p.fp32 ? 2 : 1, opts->grid_matvec > 0 ? opts->grid_matvec : p.target_slot,
                       (p.side + 1) / 2, 64);
    p.g_team = team_geom(p.side, p.S, p.B, p.target_team);
    p.g_fwd = fwd_geom(p.side, p.S, p.B, p.target_slot);
    layout(p);
    host_tables(p);
    PT_LOG(1, "plan n=%d N=%d B=%d %s%s: %d levels, workspace %.1f MiB", p.n, p.N, p.B,
           p.fp32 ? "fp32+refine" : "fp64", p.region_mode ? (p.law == PT_NU_EXPCAP ? " regions, exp-capped law" : " regions") : "",
           p.nlev, (double)p.ws_bytes / (1 << 20));
    *out = h;
    return PT_OK;
}

pt_status pt_plan_create(const pt_problem* prob, const pt_options* opts, pt_plan** out) {
    if (!prob) {
        if (out) *out = nullptr;
        return fail(PT_ERR_INVALID, "problem and options must not be NULL");
    }
    return plan_create_impl(prob, 1, opts, out);
}

pt_status pt_plan_create_batch(const pt_problem* probs, int32_t count, const pt_options* opts, pt_plan** out) {
    return plan_create_impl(probs, count, opts, out);
}

pt_status pt_plan_batch_size(const pt_plan* plan, int32_t* count) {
    if (!plan || !count) return fail(PT_ERR_INVALID, "plan and count must not be NULL");
    *count = plan->p.B;
    return PT_OK;
}

void pt_plan_destroy(pt_plan* plan) {
    if (!plan) return;
    if (plan->p.tm) {
        for (int i = 0; i < 2 * Timer::kCap; ++i) hipEventDestroy(plan->p.tm->ev[i]);
        delete plan->p.tm;
    }
    graph_release(plan->p);
    delete[] plan->p.h_tw64;
    delete[] plan->p.h_tw32;
    delete[] plan->p.h_zs;
    delete[] plan->p.h_wave;
    delete[] plan->p.h_inst;
    delete[] plan->p.h_regp;
    delete[] plan->p.h_rsj;
    delete[] plan->p.probs;
    delete plan;
}

pt_status pt_plan_check_bounds(const pt_plan* plan, char* msg, size_t cap) {
    if (!plan) return fail(PT_ERR_INVALID, "plan must not be NULL");
    std::string m;
    pt_status s = check_bounds(plan->p, m);
    if (msg && cap > 0) {
        std::snprintf(msg, cap, "%s", m.c_str());
    }
    if (s != PT_OK) return fail(s, "launch bounds: " + m);
    return PT_OK;
}

pt_status pt_plan_workspace_bytes(const pt_plan* plan, size_t* bytes) {
    if (!plan || !bytes) return fail(PT_ERR_INVALID, "plan and bytes must not be NULL");
    *bytes = plan->p.ws_bytes;
    return PT_OK;
}

pt_status pt_solve(pt_plan* plan, void* d_ws, size_t ws_bytes, double* d_u, void* stream, pt_stats* stats) {
    if (!plan || !d_u) return fail(PT_ERR_INVALID, "plan and d_u must not be NULL");
    if (plan->p.B != 1) return fail(PT_ERR_INVALID, "pt_solve takes a single-problem plan; use pt_solve_batch");
    return solve_impl(plan->p, d_ws, ws_bytes, d_u, (hipStream_t)stream, stats);
}

pt_status pt_solve_batch(pt_plan* plan, void* d_ws, size_t ws_bytes, double* d_u, void* stream, pt_stats* stats) {
    if (!plan || !d_u) return fail(PT_ERR_INVALID, "plan and d_u must not be NULL");
    return solve_impl(plan->p, d_ws, ws_bytes, d_u, (hipStream_t)stream, stats);
}

pt_status pt_solve_noalloc(pt_plan* plan, double* d_u, void* stream, pt_stats* stats) {
    if (!plan || !d_u) return fail(PT_ERR_INVALID, "plan and d_u must not be NULL");
    Plan& p = plan->p;
    if (p.opt.timing || p.opt.graph)
        return fail(PT_ERR_INVALID, "pt_solve_noalloc: options.timing and options.graph create HIP objects; "
                                    "use pt_solve / pt_solve_batch");
    if (p.ws_bytes > kScratchBytes)
        return fail(PT_ERR_WORKSPACE, "pt_solve_noalloc: the plan needs " + std::to_string(p.ws_bytes) +
                                          " bytes of workspace, more than the " + std::to_string(kScratchBytes) +
                                          " bytes of the static device scratch; use pt_solve with a workspace");
    void* ws = nullptr;
    pt_status s = scratch_address(&ws);
    if (s != PT_OK) return s;
    return solve_impl(p, ws, kScratchBytes, d_u, (hipStream_t)stream, stats, false, nullptr, true);
}

pt_status pt_residual(pt_plan* plan, void* d_ws, size_t ws_bytes, const double* d_u, double* d_r, void* stream,
                      double* rel_out, double* fnorm_out) {
    if (!plan || !d_u || !d_r) return fail(PT_ERR_INVALID, "plan, d_u and d_r must not be NULL");
    Plan& p = plan->p;
    if (p.B != 1) return fail(PT_ERR_INVALID, "component entry points take a single-problem plan");
    pt_status s = check_ws(&p, d_ws, ws_bytes);
    if (s != PT_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    char* ws = (char*)d_ws;
    s = setup(p, ws, st);
    if (s != PT_OK) return s;
    double* U = (double*)(ws + p.off_U);
    if (p.prob.d_load) launch_transpose_in(p, p.prob.d_load, (double*)(ws + p.off_F), st);
    launch_transpose_in(p, d_u, U, st);
    double* part = (double*)(ws + p.off_part);
    double* scal = (double*)(ws + p.off_scal);
    // R is first written node-major into d_r (same size), then moved through U and
    // transposed back into d_r in the time-field layout.
    const int flat = launch_forward(p, ws, TM_RESIDUAL, U, nullptr, d_r, part, st);
    launch_reduce_norms(p, ws, part, flat, scal, st);
    double h[2];
    PT_HIP(hipMemcpyAsync(h, scal, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    PT_HIP(hipStreamSynchronize(st));
    PT_HIP(hipGetLastError());
    PT_HIP(hipMemcpyAsync(U, d_r, p.nodes * p.N * sizeof(double), hipMemcpyDeviceToDevice, st));
    launch_transpose_out(p, U, d_r, st);
    PT_HIP(hipStreamSynchronize(st));
    PT_HIP(hipGetLastError());
    if (fnorm_out) *fnorm_out = std::sqrt(h[1]);
    if (rel_out) *rel_out = (h[1] > 0) ? std::sqrt(h[0] / h[1]) : std::sqrt(h[0]);
    return PT_OK;
}

pt_status pt_residual_spectrum(pt_plan* plan, void* d_ws, size_t ws_bytes, const double* d_u, void* d_rhat,
                               void* stream, double* rel_out, double* fnorm_out) {
    if (!plan || !d_u || !d_rhat) return fail(PT_ERR_INVALID, "plan, d_u and d_rhat must not be NULL");
    Plan& p = plan->p;
    if (p.B != 1) return fail(PT_ERR_INVALID, "component entry points take a single-problem plan");
    pt_status s = check_ws(&p, d_ws, ws_bytes);
    if (s != PT_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    char* ws = (char*)d_ws;
    s = setup(p, ws, st);
    if (s != PT_OK) return s;
    double* U = (double*)(ws + p.off_U);
    if (p.prob.d_load) launch_transpose_in(p, p.prob.d_load, (double*)(ws + p.off_F), st);
    launch_transpose_in(p, d_u, U, st);
    double* part = (double*)(ws + p.off_part);
    double* scal = (double*)(ws + p.off_scal);
    const int flat = launch_forward(p, ws, TM_RESIDUAL, U, d_rhat, nullptr, part, st);
    launch_reduce_norms(p, ws, part, flat, scal, st);
    double h[2];
    PT_HIP(hipMemcpyAsync(h, scal, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    PT_HIP(hipStreamSynchronize(st));
    PT_HIP(hipGetLastError());
    if (fnorm_out) *fnorm_out = std::sqrt(h[1]);
    if (rel_out) *rel_out = (h[1] > 0) ? std::sqrt(h[0] / h[1]) : std::sqrt(h[0]);
    return PT_OK;
}

pt_status pt_apply_K(pt_plan* plan, void* d_ws, size_t ws_bytes, const double* d_u, double* d_ku, int32_t nslices,
                     void* stream) {
    if (!plan || !d_u || !d_ku) return fail(PT_ERR_INVALID, "plan, d_u and d_ku must not be NULL");
    Plan& p = plan->p;
    if (p.B != 1) return fail(PT_ERR_INVALID, "component entry points take a single-problem plan");
    if (nslices < 1 || nslices > p.N) return fail(PT_ERR_INVALID, "nslices must be in [1, N]");
    pt_status s = check_ws(&p, d_ws, ws_bytes);
    if (s != PT_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    char* ws = (char*)d_ws;
    s = setup(p, ws, st);
    if (s != PT_OK) return s;
    launch_apply_K(p, ws, d_u, d_ku, nslices, st);
    PT_HIP(hipGetLastError());
    return PT_OK;
}

pt_status pt_device_reciprocals(const double* d_x, double* d_y, int64_t n, void* stream) {
    if (n < 0) return fail(PT_ERR_INVALID, "n must be >= 0");
    if (n == 0) return PT_OK;
    if (!d_x || !d_y) return fail(PT_ERR_INVALID, "d_x and d_y must not be NULL");
    launch_reciprocals(d_x, d_y, (long)n, (hipStream_t)stream);
    PT_HIP(hipGetLastError());
    return PT_OK;
}

pt_status pt_time_rfft(pt_plan* plan, void* d_ws, size_t ws_bytes, const double* d_x, void* d_xhat, void* stream) {
    if (!plan || !d_x || !d_xhat) return fail(PT_ERR_INVALID, "plan, d_x and d_xhat must not be NULL");
    Plan& p = plan->p;
    if (p.B != 1) return fail(PT_ERR_INVALID, "component entry points take a single-problem plan");
    pt_status s = check_ws(&p, d_ws, ws_bytes);
    if (s != PT_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    char* ws = (char*)d_ws;
    s = setup(p, ws, st);
    if (s != PT_OK) return s;
    double* U = (double*)(ws + p.off_U);
    launch_transpose_in(p, d_x, U, st);
    launch_forward(p, ws, TM_SIGNAL, U, d_xhat, nullptr, (double*)(ws + p.off_part), st);
    PT_HIP(hipGetLastError());
    return PT_OK;
}

pt_status pt_time_irfft(pt_plan* plan, void* d_ws, size_t ws_bytes, const void* d_xhat, double* d_x, void* stream) {
    if (!plan || !d_x || !d_xhat) return fail(PT_ERR_INVALID, "plan, d_xhat and d_x must not be NULL");
    Plan& p = plan->p;
    if (p.B != 1) return fail(PT_ERR_INVALID, "component entry points take a single-problem plan");
    pt_status s = check_ws(&p, d_ws, ws_bytes);
    if (s != PT_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    char* ws = (char*)d_ws;
    s = setup(p, ws, st);
    if (s != PT_OK) return s;
    double* U = (double*)(ws + p.off_U);
    launch_inverse(p, ws, d_xhat, nullptr, U, 0, st);
    launch_transpose_out(p, U, d_x, st);
    PT_HIP(hipGetLastError());
    return PT_OK;
}

pt_status pt_shifted_apply(pt_plan* plan, void* d_ws, size_t ws_bytes, const void* d_x, void* d_y, void* stream) {
    if (!plan || !d_x || !d_y) return fail(PT_ERR_INVALID, "plan, d_x and d_y must not be NULL");
    Plan& p = plan->p;
    if (p.B != 1) return fail(PT_ERR_INVALID, "component entry points take a single-problem plan");
    pt_status s = check_ws(&p, d_ws, ws_bytes);
    if (s != PT_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    char* ws = (char*)d_ws;
    s = setup(p, ws, st);
    if (s != PT_OK) return s;
    launch_matvec(p, ws, d_x, d_y, DOT_NONE, nullptr, st);
    PT_HIP(hipGetLastError());
    return PT_OK;
}

pt_status pt_precond_apply(pt_plan* plan, void* d_ws, size_t ws_bytes, const void* d_r, void* d_x, void* stream) {
    if (!plan || !d_r || !d_x) return fail(PT_ERR_INVALID, "plan, d_r and d_x must not be NULL");
    Plan& p = plan->p;
    if (p.B != 1) return fail(PT_ERR_INVALID, "component entry points take a single-problem plan");
    pt_status s = check_ws(&p, d_ws, ws_bytes);
    if (s != PT_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    char* ws = (char*)d_ws;
    s = setup(p, ws, st);
    if (s != PT_OK) return s;
    launch_vcycle(p, ws, d_r, d_x, DOT_NONE, nullptr, st);
    PT_HIP(hipGetLastError());
    return PT_OK;
}

pt_status pt_periodic_solve(pt_plan* plan, void* d_ws, size_t ws_bytes, const double* d_r, double* d_x,
                            int32_t inner_iters, void* stream) {
    if (!plan || !d_r || !d_x) return fail(PT_ERR_INVALID, "plan, d_r and d_x must not be NULL");
    Plan& p = plan->p;
    if (p.B != 1) return fail(PT_ERR_INVALID, "component entry points take a single-problem plan");
    if (inner_iters < 0 || inner_iters > 64) return fail(PT_ERR_INVALID, "inner_iters must be in [0, 64]");
    pt_status s = check_ws(&p, d_ws, ws_bytes);
    if (s != PT_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    char* ws = (char*)d_ws;
    s = setup(p, ws, st);
    if (s != PT_OK) return s;
    double* U = (double*)(ws + p.off_U);
    launch_transpose_in(p, d_r, U, st);
    launch_forward(p, ws, TM_SIGNAL, U, ws + p.lev[0].off_r, nullptr, (double*)(ws + p.off_part), st);
    const void* X = nullptr;
    const double* coef = nullptr;
    s = inner_solve(p, ws, st, inner_iters > 0 ? inner_iters : p.opt.inner_iters, &X, &coef);
    if (s != PT_OK) return s;
    launch_inverse(p, ws, X, coef, U, 0, st);
    launch_transpose_out(p, U, d_x, st);
    PT_HIP(hipGetLastError());
    return PT_OK;
}

pt_status pt_solve_many(int32_t count, pt_plan* const* plans, void* const* d_ws, const size_t* ws_bytes,
                        double* const* d_u, pt_stats* const* stats, pt_status* status, void* const* streams,
                        int32_t nstreams) {
    if (count < 0 || (count > 0 && (!plans || !d_ws || !ws_bytes || !d_u || !status)))
        return fail(PT_ERR_INVALID, "plans, d_ws, ws_bytes, d_u and status must not be NULL");
    if (nstreams < 1 || nstreams > 64) return fail(PT_ERR_INVALID, "nstreams must be in [1, 64]");
    for (int i = 0; i < count; ++i) {
        if (!plans[i] || !d_u[i]) return fail(PT_ERR_INVALID, "plan " + std::to_string(i) + " or its d_u is NULL");
        for (int j = 0; j < i; ++j)
            if (plans[j] == plans[i]) return fail(PT_ERR_INVALID, "a plan appears twice in the work list");
    }
    int device = 0;
    PT_HIP(hipGetDevice(&device));
    // work list: worker w takes the next unclaimed plan (in the given order) on streams[w]
    std::atomic<int> next{0};
    std::vector<std::string> errors(count);
    auto worker = [&](int w) {
        if (hipSetDevice(device) != hipSuccess) return;
        hipStream_t st = streams ? (hipStream_t)streams[w] : nullptr;
        for (int i = next.fetch_add(1); i < count; i = next.fetch_add(1)) {
            Plan& p = plans[i]->p;
            status[i] = solve_impl(p, d_ws[i], ws_bytes[i], d_u[i], st, stats ? stats[i] : nullptr);
            if (status[i] != PT_OK) errors[i] = g_last_error;
        }
    };
    for (int i = 0; i < count; ++i) status[i] = PT_ERR_INVALID;
    const int nw = std::min<int>(nstreams, std::max(count, 1));
    std::vector<std::thread> pool;
    pool.reserve(nw);
    for (int w = 0; w < nw; ++w) pool.emplace_back(worker, w);
    for (auto& th : pool) th.join();
    for (int i = 0; i < count; ++i)
        if (status[i] != PT_OK)
            return fail(status[i], "work item " + std::to_string(i) + ": " + errors[i]);
    return PT_OK;
}

pt_status pt_adjoint_solve(pt_plan* plan, void* d_ws, size_t ws_bytes, const double* d_u, double* d_lambda,
                           void* stream, pt_stats* stats) {
    if (!plan || !d_u || !d_lambda) return fail(PT_ERR_INVALID, "plan, d_u and d_lambda must not be NULL");
    Plan& p = plan->p;
    if (p.B != 1 || !p.opt.adjoint) return fail(PT_ERR_INVALID, "the plan was not created with options.adjoint = 1");
    return solve_impl(p, d_ws, ws_bytes, const_cast<double*>(d_u), (hipStream_t)stream, stats, true, d_lambda);
}

pt_status pt_loss_gradients(pt_plan* plan, void* d_ws, size_t ws_bytes, const double* d_u, const double* d_lambda,
                            double* d_gtheta, double* d_gsigma, int32_t per_cell, double* loss_out, void* stream) {
    if (!plan || !d_u) return fail(PT_ERR_INVALID, "plan and d_u must not be NULL");
    Plan& p = plan->p;
    if (p.B != 1 || !p.opt.adjoint) return fail(PT_ERR_INVALID, "the plan was not created with options.adjoint = 1");
    if (per_cell != 0 && per_cell != 1) return fail(PT_ERR_INVALID, "per_cell must be 0 or 1");
    pt_status s = check_ws(&p, d_ws, ws_bytes);
    if (s != PT_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    char* ws = (char*)d_ws;
    s = setup(p, ws, st);
    if (s != PT_OK) return s;
    launch_transpose_in(p, d_u, (double*)(ws + p.off_U), st);
    if (d_lambda) launch_transpose_in(p, d_lambda, (double*)(ws + p.off_L), st);
    launch_adj_grad(p, ws, d_lambda != nullptr, d_gtheta, d_gsigma, per_cell, st);
    double* scal = (double*)(ws + p.off_scal);
    launch_reduce_pairs(p, (const double*)(ws + p.off_part), p.n * p.n, scal, st);
    double h[2];
    PT_HIP(hipMemcpyAsync(h, scal, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    PT_HIP(hipStreamSynchronize(st));
    PT_HIP(hipGetLastError());
    if (loss_out) *loss_out = h[0];
    return PT_OK;
}

pt_status pt_newton_solve(pt_plan* plan, void* d_ws, size_t ws_bytes, double* d_u, void* stream, pt_stats* stats) {
    if (!plan || !d_u) return fail(PT_ERR_INVALID, "plan and d_u must not be NULL");
    Plan& p = plan->p;
    if (p.B != 1 || p.opt.krylov_dim < 1) return fail(PT_ERR_INVALID, "the plan was not created with options.krylov_dim > 0");
    return newton_impl(p, d_ws, ws_bytes, d_u, (hipStream_t)stream, stats);
}

pt_status pt_jacobian_apply(pt_plan* plan, void* d_ws, size_t ws_bytes, const double* d_u, const double* d_v,
                            double* d_out, int32_t transpose, void* stream) {
    if (!plan || !d_u || !d_v || !d_out) return fail(PT_ERR_INVALID, "plan, d_u, d_v and d_out must not be NULL");
    Plan& p = plan->p;
    if (p.B != 1 || !(p.opt.adjoint || p.opt.krylov_dim > 0))
        return fail(PT_ERR_INVALID, "the plan needs options.adjoint or options.krylov_dim");
    if (transpose != 0 && transpose != 1) return fail(PT_ERR_INVALID, "transpose must be 0 or 1");
    pt_status s = check_ws(&p, d_ws, ws_bytes);
    if (s != PT_OK) return s;
    hipStream_t st = (hipStream_t)stream;
    char* ws = (char*)d_ws;
    s = setup(p, ws, st);
    if (s != PT_OK) return s;
    // the state goes to the iterate buffer, v to a scratch field, J v through the second one
    double* U = (double*)(ws + p.off_U);
    double* V = (double*)(ws + (p.opt.krylov_dim > 0 ? p.off_D : p.off_L));
    double* O = (double*)(ws + (p.opt.krylov_dim > 0 ? p.off_Ut : p.off_G));
    launch_transpose_in(p, d_u, U, st);
    launch_transpose_in(p, d_v, V, st);
    launch_jac_apply(p, ws, V, nullptr, O, transpose ? -1 : +1, st);
    launch_transpose_out(p, O, d_out, st);
    PT_HIP(hipStreamSynchronize(st));
    PT_HIP(hipGetLastError());
    return PT_OK;
}

}  // extern "C"
