// Host-side check of a plan's launch geometry and workspace layout: every workgroup of every
// sweeping kernel is walked with the same range helpers the kernels use (sweep_range,
// virtual_block_of), and every index range and partial-sum slot a launch can address is compared
// with the buffer it lands in. Nothing here runs on the GPU: it is the bounds check of a CPU run,
// for tests and for callers who want to validate a plan before its first launch.
#include <algorithm>
#include <cstdio>
#include <string>
#include <vector>

#include "pt_device.h"

namespace pt {

int cocg_rows(const Plan& p);

namespace {

constexpr size_t kMaxDynLds = 65536;  // dynamic LDS a launch may ask for

struct Buf {
    const char* name;
    size_t off, bytes;
};

struct Checker {
    const Plan& p;
    std::string err;
    explicit Checker(const Plan& q) : p(q) {}
    bool fail(const std::string& m) {
        if (err.empty()) err = m;
        return false;
    }
    bool ok() const { return err.empty(); }
};

size_t dbl(size_t n) { return n * sizeof(double); }

// workspace buffers of the plan (offsets as laid out, sizes as the kernels address them)
std::vector<Buf> buffers(const Plan& p) {
    std::vector<Buf> v;
    const size_t S = p.ST, B = p.B;
    const size_t tf = p.nodes * (size_t)p.N * sizeof(double);
    v.push_back({"U", p.off_U, p.nodes * B * p.N * sizeof(double)});
    if (p.prob.d_load) v.push_back({"F", p.off_F, tf});
    for (int l = 0; l < p.nlev; ++l) {
        const LevelDesc& d = p.lev[l];
        v.push_back({"mass stencil", d.off_mt, dbl(4 * d.nodes)});
        if (p.vk) v.push_back({"Khat stencil", d.off_kt, dbl(4 * d.nodes)});
        v.push_back({"level r", d.off_r, d.nodes * S * p.elem});
        v.push_back({"level x", d.off_x, d.nodes * S * p.elem});
    }
    if (p.has_cocg_vectors) {
        const size_t vb = p.nodes * S * p.elem;
        v.push_back({"cocg x", p.off_cx, vb});
        v.push_back({"cocg r", p.off_cr, vb});
        v.push_back({"cocg q", p.off_cq, vb});
        v.push_back({"cocg p", p.off_cp, vb});
        v.push_back({"cocg norm partials", p.off_npart, dbl((size_t)(cocg_rows(p) + kReduceRows) * S * 3)});
        v.push_back({"cocg scalars", p.off_caux, 5 * S * 2 * sizeof(double) + 16});
    }
    v.push_back({"flags", p.off_flags, B * 2 * (size_t)p.n * p.n});
    v.push_back({"load", p.off_b, dbl(B * p.nodes)});
    v.push_back({"records", p.off_rec, dbl(B * p.nodes * (p.law == PT_NU_EXPCAP ? kRecDoublesExp : kRecDoubles))});
    v.push_back({"twiddles64", p.off_tw64, dbl((size_t)p.N * 2)});
    v.push_back({"twiddles32", p.off_tw32, (size_t)p.N * 2 * sizeof(float)});
    v.push_back({"shifts", p.off_zs, dbl(S * 3)});
    v.push_back({"waveform", p.off_wave, dbl(B * p.N)});
    v.push_back({"instances", p.off_inst, dbl(B * 4)});
    v.push_back({"region laws", p.off_regp, dbl(B * kMaxRegions * 4)});
    v.push_back({"region sigma/j", p.off_rsj, dbl(kMaxRegions * 2)});
    v.push_back({"region nu_hat", p.off_rkh, dbl(kMaxRegions)});
    v.push_back({"partials", p.off_part, p.part_bytes});
    v.push_back({"norms", p.off_scal, dbl(2 * B)});
    v.push_back({"flag", p.off_flag, sizeof(int)});
    if (p.opt.adjoint) {
        v.push_back({"adjoint lambda", p.off_L, tf});
        v.push_back({"adjoint source", p.off_G, tf});
        v.push_back({"triangle sigma", p.off_sig, dbl(2 * (size_t)p.n * p.n)});
    }
    if (p.opt.krylov_dim > 0) {
        const size_t m = p.opt.krylov_dim;
        v.push_back({"newton residual", p.off_R, tf});
        v.push_back({"newton trial", p.off_Ut, tf});
        v.push_back({"newton step", p.off_D, tf});
        v.push_back({"krylov basis V", p.off_V, (m + 1) * p.tf_stride});
        v.push_back({"krylov basis Z", p.off_Z, m * p.tf_stride});
    }
    v.push_back({"per-slot coefficients", p.off_coef, 8 * S * 2 * sizeof(double)});
    return v;
}

void check_layout(Checker& c) {
    const Plan& p = c.p;
    std::vector<Buf> v = buffers(p);
    for (const Buf& b : v) {
        if (b.off % 256 != 0) c.fail(std::string(b.name) + " is not 256-byte aligned");
        if (b.off + b.bytes > p.ws_bytes)
            c.fail(std::string(b.name) + " ends at " + std::to_string(b.off + b.bytes) + " beyond the workspace (" +
                   std::to_string(p.ws_bytes) + " bytes)");
    }
    std::sort(v.begin(), v.end(), [](const Buf& a, const Buf& b) { return a.off < b.off; });
    for (size_t k = 1; k < v.size(); ++k)
        if (v[k - 1].off + v[k - 1].bytes > v[k].off && v[k].bytes > 0)
            c.fail(std::string(v[k - 1].name) + " overlaps " + v[k].name);
}

// A slot-vector sweep (V-cycle, operator): every workgroup (vb, chunk) covers per_step column units
// of rows [row0, row1) plus the one-row halo (clamped onto the grid), slots chunk * slot_chunk * V
// .. + slot_chunk * V - 1. dot_rows: the rows of the partial buffer its dot partials use (0: none).
void check_slot(Checker& c, const char* what, const Geom& g, int side, int cols, int V, size_t nodes,
                size_t dot_rows) {
    const Plan& p = c.p;
    if (g.per_step * g.slot_chunk != kBlock) c.fail(std::string(what) + ": workgroup is not one full block");
    if ((size_t)g.chunks * g.slot_chunk * V != (size_t)p.ST)
        c.fail(std::string(what) + ": slot chunks do not tile the " + std::to_string(p.ST) + " slots");
    if (g.blocks % kNumXcd != 0) c.fail(std::string(what) + ": workgroups not a multiple of the XCD count");
    if ((long)g.col_groups * g.per_step < cols) c.fail(std::string(what) + ": column groups miss columns");
    if ((long)g.col_groups * ((side + g.rows_per_chunk - 1) / g.rows_per_chunk) > g.blocks)
        c.fail(std::string(what) + ": workgroups miss row chunks");
    for (int b = 0; b < g.blocks && c.ok(); ++b) {
        const int vb = virtual_block_of(b, g.blocks, p.opt.xcd_remap);
        if (vb < 0 || vb >= g.blocks) c.fail(std::string(what) + ": virtual workgroup index out of range");
        const SweepRange r = sweep_range(vb, g.col_groups, g.per_step, g.rows_per_chunk, side);
        if (r.row0 < 0 || r.row0 > r.row1 || r.row1 > side) c.fail(std::string(what) + ": row range out of the grid");
        // highest element a lane can touch (rows and columns clamped onto the grid, as the kernels do)
        const long rmax = std::min(r.row1 + 2, side - 1);
        const size_t node = (size_t)rmax * side + (side - 1);
        const size_t slot = (size_t)(g.chunks - 1) * g.slot_chunk * V + (size_t)g.slot_chunk * V - 1;
        if (node >= nodes || slot >= (size_t)p.ST) c.fail(std::string(what) + ": element index beyond the slot vector");
        if (dot_rows && (size_t)vb >= dot_rows) c.fail(std::string(what) + ": dot partial row beyond its buffer");
    }
}

// per-node team sweeps over B (n+1) virtual columns: the residual sweep (team of TS threads, KP
// pairs per lane) and the time DFTs (team of S/4 threads, two slot pairs per lane)
void check_team(Checker& c, const char* what, const Geom& g, size_t units, int team, long covered, long needed,
                size_t part_pairs) {
    const Plan& p = c.p;
    if ((long)g.per_step * team > kBlock) c.fail(std::string(what) + ": teams exceed the workgroup");
    if (team <= 0 || covered < needed) c.fail(std::string(what) + ": the team's lanes do not cover the series");
    if ((size_t)g.col_groups * g.per_step < units) c.fail(std::string(what) + ": column groups miss columns");
    for (int b = 0; b < g.blocks && c.ok(); ++b) {
        const int vb = virtual_block_of(b, g.blocks, p.opt.xcd_remap);
        const SweepRange r = sweep_range(vb, g.col_groups, g.per_step, g.rows_per_chunk, p.side);
        if (r.row0 < 0 || r.row0 > r.row1 || r.row1 > p.side) c.fail(std::string(what) + ": row range out of the grid");
        if (part_pairs && ((size_t)vb * g.per_step + (g.per_step - 1)) >= part_pairs)
            c.fail(std::string(what) + ": norm partial beyond the partial buffer");
    }
}

}  // namespace

pt_status check_bounds(const Plan& p, std::string& msg) {
    Checker c(p);
    check_layout(c);
    const int V = p.fp32 ? 2 : 1;
    const size_t part_doubles = p.part_bytes / sizeof(double);
    // slot partial sets: V-cycle dots (level 0) and the operator's, each with its stage-1 tail
    const size_t set_a = (size_t)(p.g_slot0.blocks + kReduceRows) * p.ST * 3;
    const size_t set_b = (size_t)(p.g_mv.blocks + kReduceRows) * p.ST * 3;
    if (set_a + set_b > part_doubles) c.fail("the two dot-partial sets exceed the partial buffer");
    const Geom up0 = slot_geom(p.side, p.ST, V, p.target_up);
    if (up0.blocks != p.g_slot0.blocks || up0.rows_per_chunk != p.g_slot0.rows_per_chunk)
        c.fail("level-0 up sweep geometry differs from the one its dot partials are sized for");
    check_slot(c, "V-cycle up sweep level 0", p.g_slot0, p.side, p.side, V, p.nodes, (size_t)p.g_slot0.blocks);
    check_slot(c, "operator (column pairs)", p.g_mv, p.side, (p.side + 1) / 2, V, p.nodes, (size_t)p.g_mv.blocks);
    for (int l = 1; l < p.nlev && c.ok(); ++l) {
        // the restriction into level l and the up sweep onto level l
        const Geom gd = slot_geom(p.lev[l].side, p.ST, V, p.target_down);
        check_slot(c, ("V-cycle restriction into level " + std::to_string(l)).c_str(), gd, p.lev[l].side,
                   p.lev[l].side, V, p.lev[l].nodes, 0);
        const Geom gu = slot_geom(p.lev[l].side, p.ST, V, p.target_up);
        check_slot(c, ("V-cycle up sweep level " + std::to_string(l)).c_str(), gu, p.lev[l].side, p.lev[l].side, V,
                   p.lev[l].nodes, 0);
    }
    // residual sweep: TS = min(S, 256) threads per column, norm partials two per team
    const int TS = p.S < kBlock ? p.S : kBlock;
    if (p.S / TS > 2) c.fail("residual sweep: more than two time pairs per lane");
    const size_t fwd_pairs = part_doubles / 2;
    // lane lt owns the time pairs lt + TS k, k < S / TS
    check_team(c, "residual sweep", p.g_fwd, (size_t)p.side * p.B, TS, (long)TS * (p.S / TS), p.S, fwd_pairs);
    // row buffers (or the norm reduction), plus the twiddle table where the transform is fused in
    const bool fused = p.S / TS == 1 && p.S >= 4 && p.S <= 256;
    const size_t fwd_lds = std::max((size_t)(kBlock / TS) * 4 * p.S * 4 * sizeof(double), 2 * kBlock * sizeof(double)) +
                           (fused ? (size_t)p.N * p.elem : 0);
    if (fwd_lds > kMaxDynLds) c.fail("residual sweep: LDS request above 64 KiB");
    // time DFT and inverse DFT: S/4 threads per node
    // lane lt owns the slot pairs lt and lt + TS of the S / 2 pairs
    check_team(c, "time DFT / inverse", p.g_team, (size_t)p.side * p.B, p.g_team.slot_chunk,
               2L * p.g_team.slot_chunk, p.S / 2, 0);
    if ((size_t)p.g_team.per_step * 2 * p.S * p.elem > kMaxDynLds) c.fail("time DFT: LDS request above 64 KiB");
    // COCG vector kernels and their reduction
    if (p.has_cocg_vectors) {
        const int SC = p.ST < kBlock ? p.ST : kBlock;
        if (p.ST % SC != 0) c.fail("COCG: slots not a multiple of the slot chunk");
        if (cocg_rows(p) < 1 || cocg_rows(p) > kCocgRows) c.fail("COCG: row count out of range");
    }
    // the levels the small-level kernel holds in LDS
    size_t small = 0;
    for (int l = 1; l < p.nlev; ++l)
        if (p.lev[l].side <= 33) {
            for (int q = l; q < p.nlev; ++q) small += 2 * p.lev[q].nodes;
            small += p.lev[l].nodes;
            break;
        }
    if (small * p.elem > kMaxDynLds) c.fail("small-level V-cycle: LDS request above 64 KiB");
    if (p.opt.adjoint && part_doubles < std::max<size_t>(2 * kAdjBlocks, 2 * (size_t)p.n * p.n))
        c.fail("adjoint: partial buffer too small");
    if (p.opt.krylov_dim > 0 && part_doubles < 2 * (size_t)kAdjBlocks) c.fail("Krylov dots: partial buffer too small");
    msg = c.err;
    return c.ok() ? PT_OK : PT_ERR_INVALID;
}

}  // namespace pt
