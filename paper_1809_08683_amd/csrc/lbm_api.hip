// Host runtime and C ABI (include/lbm.h) of the gfx950 lattice Boltzmann
// library: parameter validation and derived constants, device memory, the
// per-step work list, launches, reductions and checkpoints.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <tuple>
#include <mutex>
#include <string>
#include <vector>

#include "lbm.h"
#include "lbm_launch.hpp"
#include "lbm_params.hpp"
#include "lbm_rounding.hpp"


namespace {

constexpr double kCs2 = 1.0 / 3.0;
// model constants of Sec. 4 used on the host side (rest state, kappa)
constexpr double kVarpi = 1.0 / 6.0, kGamma1 = -2.0, kGamma2 = 2.0;
constexpr double kKappa = 2.0 / 3.0 + kGamma1 / 2.0 + kGamma2 / 3.0;
constexpr int kRedBlocks = 240;
// Per-case flag area (256 bytes after the macro arrays): the divergence flag
// at byte 0, the two step counters of the stochastic rounding at byte 64.
constexpr size_t kTickOffset = 64;

// bytes of one f value and of one g value as stored
size_t f_size(int prec) { return prec == LBM_FP64 ? 8 : (prec == LBM_FP16S ? 2 : 4); }
size_t g_size(int prec) { return prec == LBM_FP64 ? 8 : (prec == LBM_FP32 ? 4 : 2); }
size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

struct Layout {
    int pitch;
    long long plane;
    size_t buf_bytes, macro_bytes, flag_bytes, total;
};

Layout layout_of(int nx, int ny, int prec)
{
    Layout L;
    // enough 64-slot strip regions for the off-wall columns of either kind of
    // x boundary (periodic needs ceil(nx / 62), walled ceil((nx - 2) / 62)),
    // plus at least two regions that hold at most the right ghost column and,
    // in the row's last slot, the left one, rounded up to an odd count: the
    // row stride is then an odd multiple of a region, and the rows a step
    // touches at once fall on the HBM channels more evenly (on the 2048^2
    // cavity 36 regions ran FP32 3 % and FP64 4 % slower than 37; pads from 2
    // to 11 regions spanned 4 % in FP32 and 10 % in FP64).
    const int regions = (nx + lbm::STRIP_COLS - 1) / lbm::STRIP_COLS + 2;
    L.pitch = (regions | 1) * lbm::REGION_SLOTS;
    L.plane = (long long)(ny + 2) * L.pitch;
    L.buf_bytes = round_up(size_t(9) * L.plane * (f_size(prec) + g_size(prec)), 256);
    L.macro_bytes = round_up(size_t(5) * nx * ny * sizeof(double), 256);
    L.flag_bytes = 256;
    L.total = 2 * L.buf_bytes + L.macro_bytes + L.flag_bytes;
    return L;
}

struct CaseHost {
    int nx, ny;
    Layout L;
    char* base = nullptr;     // start of the case's device memory
    bool inited = false;
    long long diverged_at = -1;   // t at the end of the step call that first saw the case diverged
};

}  // namespace

struct lbm_ctx {
    int prec = LBM_FP32;
    std::vector<lbm::CaseParams> P;
    std::vector<CaseHost> H;
    lbm::CaseParams* d_P = nullptr;
    std::vector<lbm::WorkItem> work;     // one entry per wavefront slot of the launch
    lbm::WorkItem* d_work = nullptr;
    size_t d_work_cap = 0;               // entries d_work can hold
    int seg_rows = 0;                    // rows per interior item (0: automatic)
    // launch configuration: kernel variant and work-list settings (lbm_autotune)
    int variant = 0;
    double xw_scale = 1.0;
    int bands_per_xcd = 4;
    // instantiated graphs of n steps, by (n, start parity, persistent);
    // dropped when the launch configuration changes
    std::map<std::tuple<long long, int, int>, hipGraphExec_t> graphs;
    // persistent stepping (lbm_step_ex with LBM_STEP_PERSISTENT): per-case
    // arrival counters, the abort word and per-case wavefront counts, set up
    // with the work list; the launch is allowed only if its blocks are all
    // resident at once
    unsigned* d_pcount = nullptr;
    int* d_pabort = nullptr;
    int* d_case_arrivals = nullptr;
    bool persistent_ok = false;
    std::string persistent_why;
    unsigned spin_limit = 1u << 24;      // polls of a persistent step barrier before it gives up
    long long n_items = 0;               // non-empty entries
    double* d_red = nullptr;
    std::vector<void*> allocs;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int device = 0;                      // device current at creation
    int parity = 0;
    long long t = 0;
    std::string err;
};

namespace {

lbm_status fail(lbm_ctx* c, lbm_status code, const std::string& msg)
{
    if (c) c->err = msg;
    return code;
}

lbm_status hip_fail(lbm_ctx* c, hipError_t e, const char* where)
{
    return fail(c, LBM_EDEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

#define HIP_TRY(ctx, expr)                                             \
    do {                                                               \
        hipError_t e_ = (expr);                                        \
        if (e_ != hipSuccess) return hip_fail((ctx), e_, #expr);       \
    } while (0)

// ---- thermodynamics of the case (Sec. 4) --------------------------------
double cs_b_of(const lbm_eos& e) { return e.b > 0 ? e.b : std::sqrt(2.0) * M_PI / (3.0 * e.rho0); }

double cs_Z(double y) { return (1 + y + y * y - y * y * y) / std::pow(1 - y, 3); }

double pressure(const lbm_eos& e, double R, double rho, double T)
{
    switch (e.kind) {
    case LBM_EOS_DECOUPLED: return rho * R * e.T0;
    case LBM_EOS_IDEAL: return rho * R * T;
    case LBM_EOS_VDW: return rho * R * T / (1 - e.b * rho) - e.a * rho * rho;
    default: return cs_Z(cs_b_of(e) * rho / 4) * rho * R * T;
    }
}

// R with dp/drho(rho0, T0) = c_s^2 (eq. cs)
double gas_constant(const lbm_eos& e)
{
    if (e.R > 0) return e.R;
    switch (e.kind) {
    case LBM_EOS_DECOUPLED:
    case LBM_EOS_IDEAL: return kCs2 / e.T0;
    case LBM_EOS_VDW: return (kCs2 + 2 * e.a * e.rho0) * (1 - e.b * e.rho0) * (1 - e.b * e.rho0) / e.T0;
    default: {
        const double y = cs_b_of(e) * e.rho0 / 4;
        const double dzdy = (4 + 4 * y - 2 * y * y) / std::pow(1 - y, 4);
        return kCs2 / (e.T0 * (cs_Z(y) + y * dzdy));
    }
    }
}

template <typename C>
void fill_coef(lbm::Coef<C>& K, const lbm_eos& e, double R, double cp, double cv, double Pr,
               const lbm_relax& r, const lbm_options& o, const lbm_boundary& bc)
{
    K.rho0 = C(e.rho0);
    K.T0 = C(e.T0);
    K.inv_T0 = C(1.0 / e.T0);
    K.R = C(R);
    K.a_vdw = C(e.a);
    K.b_vdw = C(e.b);
    K.b_cs = C(cs_b_of(e));
    K.rho0_cp = C(e.rho0 * cp);
    K.mu0 = C(e.rho0 * r.nu0);
    K.suth_S = C(r.sutherland_S);
    K.suth_1pS = C(1.0 + r.sutherland_S);
    K.bulk_over_varpi = C(r.bulk_ratio / kVarpi);
    K.varpi_over_bulk = C(kVarpi / r.bulk_ratio);
    K.inv_kappa_rho0_Pr = C(1.0 / (kKappa * e.rho0 * Pr));
    K.kappa_rho0_Pr = C(kKappa * e.rho0 * Pr);
    K.fx = C(o.fx);
    K.fy = C(o.fy);
    for (int s = 0; s < 4; ++s) {
        K.side_ux[s] = C(bc.side[s].ux);
        K.side_uy[s] = C(bc.side[s].uy);
        K.side_T[s] = bc.side[s].T;
    }
    K.cv_d = cv;
    K.inv_cv_d = 1.0 / cv;
    K.rho0_d = e.rho0;
    K.T0_d = e.T0;
    K.p0_d = pressure(e, R, e.rho0, e.T0);
    K.rhoE0_d = e.rho0 * cv * e.T0;
    K.R_d = R;
    K.a_d = e.a;
    K.b_d = e.b;
    K.bcs_d = cs_b_of(e);
}

lbm_status validate(lbm_ctx* c, int nx, int ny, const lbm_eos* eos, double Pr, double gamma,
                    const lbm_relax* relax, const lbm_boundary* bc, const lbm_options* opt)
{
    if (!eos || !relax || !bc || !opt) return fail(c, LBM_EINVAL, "null parameter block");
    if (nx < 1 || ny < 1) return fail(c, LBM_EINVAL, "grid size must be positive");
    if ((long long)nx * ny > (1LL << 31) - 1) return fail(c, LBM_EINVAL, "grid too large");
    if (nx > (1 << 23)) return fail(c, LBM_EINVAL, "grid too wide (a stored row block must stay below 2 GiB)");
    if (bc->side[0].wall != bc->side[1].wall || bc->side[2].wall != bc->side[3].wall)
        return fail(c, LBM_EINVAL, "opposite sides must both be walls or both periodic");
    if ((bc->side[0].wall && nx < 5) || (bc->side[2].wall && ny < 5))
        return fail(c, LBM_EINVAL, "a walled axis needs at least 5 nodes");
    if (eos->kind < 0 || eos->kind > 3) return fail(c, LBM_EINVAL, "unknown EOS");
    if (!(eos->rho0 > 0) || !(eos->T0 > 0)) return fail(c, LBM_EINVAL, "rho0 and T0 must be positive");
    if (eos->kind == LBM_EOS_VDW && !(eos->b * eos->rho0 < 1)) return fail(c, LBM_EINVAL, "van der Waals b rho0 >= 1");
    if (!(Pr > 0) || !(gamma > 0)) return fail(c, LBM_EINVAL, "Pr and gamma must be positive");
    if (!(relax->nu0 > 0)) return fail(c, LBM_EINVAL, "nu0 must be positive");
    if (!(relax->bulk_ratio > 0)) return fail(c, LBM_EINVAL, "bulk_ratio must be positive");
    if (relax->law < 0 || relax->law > 2) return fail(c, LBM_EINVAL, "unknown viscosity law");
    if (relax->law == LBM_VISC_SUTHERLAND && !(relax->sutherland_S >= 0))
        return fail(c, LBM_EINVAL, "Sutherland S must be >= 0");
    if (bc->extrap_order < 1 || bc->extrap_order > 2) return fail(c, LBM_EINVAL, "extrap_order must be 1 or 2");
    if (opt->prec < 0 || opt->prec > 3) return fail(c, LBM_EINVAL, "unknown precision");
    if (opt->cubic < 0 || opt->cubic > 2) return fail(c, LBM_EINVAL, "cubic must be 0, 1 or 2");
    for (int s = 0; s < 4; ++s) {
        const lbm_side& sd = bc->side[s];
        if (!std::isfinite(sd.ux) || !std::isfinite(sd.uy)) return fail(c, LBM_EINVAL, "non-finite wall velocity");
        if (sd.wall && !sd.adiabatic && !(sd.T > 0)) return fail(c, LBM_EINVAL, "wall temperature must be positive");
    }
    const double R = gas_constant(*eos);
    if (!(R > 0) || !std::isfinite(R)) return fail(c, LBM_EINVAL, "equation of state gives no valid R");
    const double cp = opt->cp > 0 ? opt->cp : 3.5 * kCs2 / eos->T0;
    const double cv = opt->cv_rule ? cp - pressure(*eos, R, eos->rho0, eos->T0) / (eos->rho0 * eos->T0) : cp / gamma;
    if (!(cv > 0)) return fail(c, LBM_EINVAL, "C_v must be positive");
    return LBM_OK;
}

// whether a case's 16-bit g rows are stored relative to the conduction state
bool gref_applies(const lbm_eos& e, const lbm_boundary& bc)
{
    return e.kind == LBM_EOS_IDEAL && bc.side[0].wall && !bc.side[0].adiabatic && !bc.side[1].adiabatic;
}

void build_case(lbm::CaseParams& P, int nx, int ny, const lbm_eos& e, double Pr, double gamma,
                const lbm_relax& r, const lbm_boundary& bc, const lbm_options& o, const Layout& L,
                char* base)
{
    std::memset(&P, 0, sizeof P);
    P.nx = nx;
    P.ny = ny;
    P.pitch = L.pitch;
    P.rowblk = 18LL * L.pitch;
    P.wall_x = bc.side[0].wall ? 1 : 0;
    P.wall_y = bc.side[2].wall ? 1 : 0;
    P.xlo = P.wall_x;
    P.nstrips = (nx - 2 * P.wall_x + lbm::STRIP_COLS - 1) / lbm::STRIP_COLS;
    P.eos = e.kind;
    P.visc_law = r.law;
    P.per_mass = o.per_mass ? 1 : 0;
    P.cubic = o.cubic;
    P.extrap_order = bc.extrap_order;
    for (int s = 0; s < 4; ++s) P.side_adiabatic[s] = bc.side[s].adiabatic ? 1 : 0;
    // the buffers start 256-byte aligned and a row is a whole number of 64-slot
    // regions, so every strip region starts on a 128-byte cache line
    P.buf[0] = base;
    P.buf[1] = base + L.buf_bytes;
    P.macro = reinterpret_cast<double*>(base + 2 * L.buf_bytes);
    P.flag = reinterpret_cast<int*>(base + 2 * L.buf_bytes + L.macro_bytes);
    P.tick = reinterpret_cast<unsigned*>(base + 2 * L.buf_bytes + L.macro_bytes + kTickOffset);

    const double R = gas_constant(e);
    const double cp = o.cp > 0 ? o.cp : 3.5 * kCs2 / e.T0;
    const double cv = o.cv_rule ? cp - pressure(e, R, e.rho0, e.T0) / (e.rho0 * e.T0) : cp / gamma;
    fill_coef<double>(P.cd, e, R, cp, cv, Pr, r, o, bc);
    fill_coef<float>(P.cf, e, R, cp, cv, Pr, r, o, bc);
    // 16-bit g rows store offsets from the rest equilibrium of the conduction
    // state between two Dirichlet x-walls (ideal gas: T_ref linear from side 0
    // at x = 0 to side 1 at x = nx - 1, rho_ref T_ref = rho0 T0),
    // s(x) = rho0 C_p (T_ref(x) - T0)
    if ((o.prec == LBM_F32G16 || o.prec == LBM_FP16S) && gref_applies(e, bc)) {
        const double s0 = e.rho0 * cp * (bc.side[0].T - e.T0);
        const double k = e.rho0 * cp * (bc.side[1].T - bc.side[0].T) / double(nx - 1);
        P.cd.gs0 = s0;
        P.cd.gsk = k;
        P.cf.gs0 = float(s0);
        P.cf.gsk = float(k);
    }
}

// Work decomposition of one step.  The off-wall region of every case is cut
// into strips of 62 columns and each strip into segments of nearly equal
// height; by default the number of segments is chosen so that all items of
// a step are resident at once (one round of wavefronts).  Where the format
// allows it, the strips next to an x-wall also collide its nodes (with
// shorter segments, as their rows cost more); the other wall nodes go to
// wall items, split over wavefronts in proportion to their cost.  Without
// lockstep the wall wavefronts are spread one per block, beside interior
// ones, so that the CUs carry a similar mix of wall and interior work; with
// lockstep the wall wavefronts fill blocks of their own.  Block b runs on XCD b % 8; the
// interior items of a few contiguous bands of rows go to the blocks of one
// XCD, neighbouring strips of a segment sharing a block.
bool build_work(lbm_ctx* c, int seg_rows, int cus, int blocks_per_cu, int PB, bool lockstep, bool xw_strips,
                double xw_cost, int bands_per_xcd)
{
    constexpr int NX = 8;
    const int nc = int(c->P.size());
    const long long nblocks = (long long)round_up(size_t(std::max(cus, 1)) * size_t(std::max(blocks_per_cu, 1)), NX);
    const long long capacity = nblocks * PB;
    std::vector<int> nwall(nc, 0);
    long long total_wall = 0, total_cells = 0;   // wall nodes, strip-rows over all cases
    for (int k = 0; k < nc; ++k) {
        const auto& P = c->P[k];
        if (P.wall_y) nwall[k] += 2 * P.nx;
        if (P.wall_x && !xw_strips) nwall[k] += 2 * (P.wall_y ? P.ny - 2 : P.ny);
        total_wall += nwall[k];
        const int xr = P.wall_x ? P.nx - 2 : P.nx, yr = P.wall_y ? P.ny - 2 : P.ny;
        total_cells += (long long)((xr + lbm::STRIP_COLS - 1) / lbm::STRIP_COLS) * yr;
    }
    std::vector<lbm::WorkItem> wall;
    if (total_wall > 0) {
        // A wall node costs about kWallCost interior nodes (its own pull, the
        // pulls at x_f, x_ff along the inner normal and of its gradient
        // neighbours, the inversions).  A wavefront takes wall nodes 64 at a
        // time, in chunks of whole passes, as many as make a wall item last
        // about as long as an interior item.  Where wall items also take
        // x-wall columns (one cache line per node and DF row, gathered), a
        // pass costs about kColumnFactor times more: the gathers need many
        // wavefronts in flight (a 2048^2 FP64 cavity then gets one pass per
        // wall wavefront).
        constexpr double kWallCost = 12.0, kColumnFactor = 2.5;
        bool columns = false;
        for (int k = 0; k < nc; ++k) columns = columns || (c->P[k].wall_x && !xw_strips);
        const double pass_rows = kWallCost * lbm::REGION_SLOTS / lbm::STRIP_COLS * (columns ? kColumnFactor : 1.0);
        const double item_rows = (double(total_cells) + pass_rows * double(total_wall) / lbm::REGION_SLOTS) /
                                 double(capacity);
        const long long passes = std::max<long long>(1, std::llround(item_rows / pass_rows));
        const int chunk = int(passes * lbm::REGION_SLOTS);
        for (int k = 0; k < nc; ++k)
            for (int b = 0; b < nwall[k]; b += chunk) wall.push_back({k, 1, b, 0, std::min(chunk, nwall[k] - b), 0});
    }
    // Wall item i goes to slot i / nblocks of block i % nblocks (one per block
    // first, spreading them over the CUs).  When interior waves march in
    // lockstep, a block must not mix them with wall waves: wall items then
    // fill whole blocks of their own, spread over the XCDs.
    std::vector<int> used(size_t(nblocks), 0);
    std::vector<std::pair<long long, lbm::WorkItem>> wall_placed;
    for (size_t i = 0; i < wall.size(); ++i) {
        long long blk = lockstep ? (long long)(i / PB) : (long long)i % nblocks;
        while (blk < (long long)used.size() && used[size_t(blk)] >= PB) ++blk;
        while (blk >= (long long)used.size()) used.push_back(0);
        wall_placed.push_back({blk * PB + used[size_t(blk)], wall[i]});
        ++used[size_t(blk)];
    }
    if (lockstep)
        for (auto& u : used)
            if (u > 0) u = PB;
    const long long wall_blocks = (long long)used.size();

    // Interior items in (case, first row, strip) order; the edge strips of a
    // walled-x case (first and last) also collide the x-wall nodes, so a row
    // of theirs costs xw_cost plain rows.
    struct Cand {
        lbm::WorkItem w;
        double cost;
        bool edge;
    };
    // Segment counts for a bound T on the cost (rows, times xw_cost on edge
    // strips) of one item: every strip is cut into ceil(cost / T) segments
    // (at least 4 rows each, 2 on edge strips).
    auto seg_counts = [&](int k, double T, int& nseg, int& nseg_e) {
        const auto& P = c->P[k];
        const int rows = P.wall_y ? P.ny - 2 : P.ny;
        if (seg_rows > 0) {
            nseg = nseg_e = (rows + seg_rows - 1) / seg_rows;
            return;
        }
        nseg = std::min(std::max(1, int(std::ceil(rows / T))), std::max(1, rows / 4));
        nseg_e = std::min(std::max(1, int(std::ceil(xw_cost * rows / T))), std::max(1, rows / 2));
    };
    auto make_items = [&](double T) {
        std::vector<Cand> items;
        for (int k = 0; k < nc; ++k) {
            const auto& P = c->P[k];
            const int xlo = P.wall_x, ylo = P.wall_y;
            const int rows = P.wall_y ? P.ny - 2 : P.ny, strips = P.nstrips;
            auto is_edge = [&](int st) { return xw_strips && P.wall_x && (st == 0 || st == strips - 1); };
            int nseg, nseg_e;
            seg_counts(k, T, nseg, nseg_e);
            const size_t first = items.size();
            for (int st = 0; st < strips; ++st) {
                const bool e = is_edge(st);
                const int n = e ? nseg_e : nseg;
                for (int g = 0; g < n; ++g) {
                    const int y0 = ylo + int((long long)rows * g / n);
                    const int y1 = ylo + int((long long)rows * (g + 1) / n);
                    if (y1 <= y0) continue;
                    items.push_back({{k, 0, xlo + lbm::STRIP_COLS * st, y0, y1 - y0, g & 1},
                                     double(y1 - y0) * (e ? xw_cost : 1.0), e});
                }
            }
            std::stable_sort(items.begin() + first, items.end(), [](const Cand& a, const Cand& b) {
                return a.w.y0 != b.w.y0 ? a.w.y0 < b.w.y0 : a.w.x0 < b.w.x0;
            });
        }
        return items;
    };
    // The items are cut by their cost midpoints into kBands bands of equal
    // cost, each a contiguous run of rows; band j goes to XCD j % 8, whose
    // items fill the free slots of its blocks k, k + 8, ...  (Four bands per
    // XCD measured 0.6-1.7 % faster than one in FP32 and the same in the
    // other formats; the autotuner tries both.)  With lockstep an XCD's edge items first fill blocks
    // of their own, as their rows take longer; without it they are spaced
    // evenly among its other items.  Blocks past the resident count are
    // added if an XCD needs them.  Returns the blocks the launch needs.
    const int kBands = std::max(1, bands_per_xcd) * NX;
    auto place = [&](const std::vector<Cand>& items, std::vector<std::pair<long long, lbm::WorkItem>>* out) {
        double total_cost = 0.0;
        for (const auto& it : items) total_cost += it.cost;
        std::vector<std::vector<size_t>> on_xcd(NX);   // item indices per XCD
        double acc = 0.0;
        for (size_t i = 0; i < items.size(); ++i) {
            const double mid = acc + 0.5 * items[i].cost;
            acc += items[i].cost;
            const int j = std::min(kBands - 1, int(mid / std::max(total_cost, 1e-300) * kBands));
            const int k = j % NX;
            on_xcd[size_t(k)].push_back(i);
        }
        long long total_blocks = (long long)round_up(size_t(wall_blocks), NX);
        for (int k = 0; k < NX; ++k) {
            long long blk = k;
            int fill = blk < wall_blocks ? used[size_t(blk)] : 0;
            auto put = [&](const lbm::WorkItem& w) {
                while (fill >= PB) {
                    blk += NX;
                    fill = blk < wall_blocks ? used[size_t(blk)] : 0;
                }
                if (out) out->push_back({blk * PB + fill, w});
                ++fill;
                total_blocks = std::max(total_blocks, (blk / NX + 1) * NX);
            };
            if (lockstep) {
                for (size_t i : on_xcd[size_t(k)])
                    if (items[i].edge) put(items[i].w);
                if (fill > 0) fill = PB;   // blocks of edge items hold nothing else
                for (size_t i : on_xcd[size_t(k)])
                    if (!items[i].edge) put(items[i].w);
            } else {
                // edge items spread evenly through the band, so that no CU
                // holds more than its share of their heavier rows
                std::vector<size_t> e_i, r_i;
                for (size_t i : on_xcd[size_t(k)]) (items[i].edge ? e_i : r_i).push_back(i);
                const size_t N = e_i.size() + r_i.size(), E = e_i.size();
                size_t ie = 0, ir = 0;
                for (size_t p = 0; p < N; ++p) {
                    const bool take_e = ie < E && (ir >= r_i.size() || (2 * ie + 1) * N <= (2 * p + 1) * E);
                    put(items[take_e ? e_i[ie++] : r_i[ir++]].w);
                }
            }
        }
        return total_blocks;
    };
    // The smallest T whose items all fit the resident blocks (one round of
    // wavefronts): the longest item, which sets the step time, is then as
    // short as the device allows.
    double T = 1.0;
    if (seg_rows <= 0) {
        double lo = 0.5, hi = 1.0;
        for (int k = 0; k < nc; ++k) hi = std::max(hi, xw_cost * double(c->P[k].ny));
        auto fits = [&](double t) { return place(make_items(t), nullptr) <= nblocks; };
        if (fits(hi)) {
            for (int it = 0; it < 40; ++it) {
                const double mid = 0.5 * (lo + hi);
                (fits(mid) ? hi : lo) = mid;
            }
        }
        T = hi;
    }
    const std::vector<Cand> items = make_items(T);
    std::vector<std::pair<long long, lbm::WorkItem>> placed = wall_placed;
    const long long total_blocks = place(items, &placed);
    c->work.assign(size_t(total_blocks * PB), lbm::WorkItem{0, 2, 0, 0, 0, 0});
    for (const auto& pr : placed) {
        if (pr.first < 0 || pr.first >= (long long)c->work.size() || c->work[size_t(pr.first)].kind != 2) return false;
        c->work[size_t(pr.first)] = pr.second;
    }
    c->n_items = (long long)(wall.size() + items.size());
    return true;
}

void drop_graphs(lbm_ctx* c)
{
    for (auto& g : c->graphs) (void)hipGraphExecDestroy(g.second);
    c->graphs.clear();
}

// Sets the launch configuration: step kernel variant, edge-strip cost scale
// and row bands per XCD; rebuilds and uploads the work list for them.
lbm_status configure(lbm_ctx* c, int variant, double xw_scale, int bands_per_xcd)
{
    if (variant < 0 || variant >= lbm::NUM_STEP_VARIANTS) return fail(c, LBM_EINVAL, "unknown kernel variant");
    if (!(xw_scale > 0) || bands_per_xcd < 1) return fail(c, LBM_EINVAL, "bad work-list setting");
    lbm::StepShape sh{};
    const int e = lbm::step_shape(c->prec, variant, &sh);
    if (e != 0) return hip_fail(c, hipError_t(e), "step kernel occupancy");
    int cus = 0;
    HIP_TRY(c, hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, c->device));
    if (!build_work(c, c->seg_rows, cus, sh.blocks_per_cu, sh.block_waves, sh.lockstep != 0, sh.xw_strips != 0,
                    sh.xw_cost * xw_scale, bands_per_xcd))
        return fail(c, LBM_EDEVICE, "internal error: inconsistent work list");
    if (c->work.size() > c->d_work_cap) {
        if (c->d_work) {
            HIP_TRY(c, hipStreamSynchronize(c->stream));
            HIP_TRY(c, hipFree(c->d_work));
            c->d_work = nullptr;
            c->d_work_cap = 0;
        }
        void* p = nullptr;
        if (hipMalloc(&p, sizeof(lbm::WorkItem) * c->work.size()) != hipSuccess)
            return fail(c, LBM_ENOMEM, "hipMalloc of the work list failed");
        c->d_work = static_cast<lbm::WorkItem*>(p);
        c->d_work_cap = c->work.size();
    }
    HIP_TRY(c, hipMemcpyAsync(c->d_work, c->work.data(), sizeof(lbm::WorkItem) * c->work.size(),
                              hipMemcpyHostToDevice, c->stream));
    // persistent stepping: arrivals per step of each case (one per block
    // that holds an item of it), and whether all blocks of the persistent
    // kernel are resident at once
    const int nc = int(c->P.size());
    std::vector<int> arrivals(size_t(nc), 0);
    const size_t bw = size_t(std::max(sh.block_waves, 1));
    for (size_t b0 = 0; b0 < c->work.size(); b0 += bw) {
        std::vector<int> seen;
        for (size_t k = b0; k < std::min(b0 + bw, c->work.size()); ++k) {
            const lbm::WorkItem& w = c->work[k];
            if (w.kind == 2 || std::find(seen.begin(), seen.end(), w.case_id) != seen.end()) continue;
            seen.push_back(w.case_id);
            ++arrivals[size_t(w.case_id)];
        }
    }
    if (!c->d_case_arrivals) {
        void* p1 = nullptr;
        void* p2 = nullptr;
        void* p3 = nullptr;
        if (hipMalloc(&p1, sizeof(int) * size_t(nc)) != hipSuccess || hipMalloc(&p2, sizeof(unsigned) * size_t(nc)) != hipSuccess ||
            hipMalloc(&p3, 256) != hipSuccess) {
            if (p1) (void)hipFree(p1);
            if (p2) (void)hipFree(p2);
            return fail(c, LBM_ENOMEM, "hipMalloc of the persistent-step words failed");
        }
        c->d_case_arrivals = static_cast<int*>(p1);
        c->d_pcount = static_cast<unsigned*>(p2);
        c->d_pabort = static_cast<int*>(p3);
    }
    HIP_TRY(c, hipMemcpyAsync(c->d_case_arrivals, arrivals.data(), sizeof(int) * size_t(nc), hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    int pbpc = 0;
    const int pe = lbm::persistent_blocks(c->prec, variant, &pbpc);
    const long long blocks = (long long)(c->work.size() / size_t(std::max(sh.block_waves, 1)));
    c->persistent_ok = pe == 0 && blocks <= (long long)pbpc * cus;
    c->persistent_why = pe != 0 ? std::string("persistent kernel occupancy query failed")
                                : "the work list needs " + std::to_string(blocks) + " blocks, more than the " +
                                      std::to_string((long long)pbpc * cus) + " the persistent kernel keeps resident";
    drop_graphs(c);
    c->variant = variant;
    c->xw_scale = xw_scale;
    c->bands_per_xcd = bands_per_xcd;
    return LBM_OK;
}

lbm_status create_impl(int ncases, const int* nx, const int* ny, const lbm_eos* eos, const double* Pr,
                       const double* gamma, const lbm_relax* relax, const lbm_boundary* bc,
                       const lbm_options* opt, void* dev_ws, size_t ws_bytes, lbm_ctx** out)
{
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    lbm_ctx* c = new lbm_ctx();
    *out = c;
    if (ncases < 1) return fail(c, LBM_EINVAL, "ncases must be >= 1");
    if (!nx || !ny || !eos || !Pr || !gamma || !relax || !bc || !opt)
        return fail(c, LBM_EINVAL, "null parameter block");
    c->prec = opt[0].prec;
    lbm_status st = LBM_OK;
    for (int k = 0; k < ncases; ++k) {
        st = validate(c, nx[k], ny[k], &eos[k], Pr[k], gamma[k], &relax[k], &bc[k], &opt[k]);
        if (st != LBM_OK) return st;
        if (opt[k].prec != c->prec) return fail(c, LBM_EINVAL, "all cases of a batch share one precision");
    }
    HIP_TRY(c, hipGetDevice(&c->device));
    // device memory
    size_t total = 0;
    std::vector<Layout> L(ncases);
    for (int k = 0; k < ncases; ++k) {
        L[k] = layout_of(nx[k], ny[k], c->prec);
        total += L[k].total;
    }
    char* base = nullptr;
    if (dev_ws) {
        if (ws_bytes < total) return fail(c, LBM_ENOMEM, "workspace smaller than lbm_workspace_bytes");
        if (reinterpret_cast<uintptr_t>(dev_ws) % 256) return fail(c, LBM_EINVAL, "workspace must be 256-byte aligned");
        base = static_cast<char*>(dev_ws);
    } else {
        void* p = nullptr;
        if (hipMalloc(&p, total) != hipSuccess) return fail(c, LBM_ENOMEM, "hipMalloc of the lattice failed");
        c->allocs.push_back(p);
        base = static_cast<char*>(p);
    }
    if (opt[0].hip_stream) {
        c->stream = static_cast<hipStream_t>(opt[0].hip_stream);
    } else {
        HIP_TRY(c, hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
        c->own_stream = true;
    }
    HIP_TRY(c, hipMemsetAsync(base, 0, total, c->stream));
    c->P.resize(ncases);
    c->H.resize(ncases);
    size_t off = 0;
    for (int k = 0; k < ncases; ++k) {
        build_case(c->P[k], nx[k], ny[k], eos[k], Pr[k], gamma[k], relax[k], bc[k], opt[k], L[k], base + off);
        c->H[k].nx = nx[k];
        c->H[k].ny = ny[k];
        c->H[k].L = L[k];
        c->H[k].base = base + off;
        off += L[k].total;
    }
    void* p = nullptr;
    HIP_TRY(c, hipMalloc(&p, sizeof(lbm::CaseParams) * ncases));
    c->allocs.push_back(p);
    c->d_P = static_cast<lbm::CaseParams*>(p);
    c->seg_rows = opt[0].seg_rows;
    st = configure(c, 0, 1.0, 4);
    if (st != LBM_OK) return st;
    HIP_TRY(c, hipMalloc(&p, sizeof(double) * (kRedBlocks * 4 + 8)));
    c->allocs.push_back(p);
    c->d_red = static_cast<double*>(p);
    HIP_TRY(c, hipMemcpyAsync(c->d_P, c->P.data(), sizeof(lbm::CaseParams) * ncases, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status check_ctx(lbm_ctx* c)
{
    if (!c) return LBM_EINVAL;
    if (c->P.empty()) return fail(c, LBM_ESTATE, "context was not created successfully");
    return LBM_OK;
}

lbm_status check_case(lbm_ctx* c, int k)
{
    lbm_status st = check_ctx(c);
    if (st != LBM_OK) return st;
    if (k < 0 || k >= int(c->P.size())) return fail(c, LBM_EINVAL, "case index out of range");
    return LBM_OK;
}

lbm_status read_flags(lbm_ctx* c, std::vector<int>& flags)
{
    flags.assign(c->P.size(), 0);
    for (size_t k = 0; k < c->P.size(); ++k)
        HIP_TRY(c, hipMemcpyAsync(&flags[k], c->P[k].flag, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

// Checkpoint layout: an 8-byte format tag, t and the case count, one
// CkptCase record per case, then per case the current DF buffer and the
// macro array.  lbm_load accepts a checkpoint only if every record equals the
// context's own.  The record includes the reference of 16-bit g rows
// (zero without one), which the stored bits are measured from.
constexpr char kCkptMagic[8] = {'L', 'B', 'M', 'C', 'K', 'P', 'T', '4'};
constexpr size_t kCkptHeader = 24;
struct CkptCase {
    int nx, ny, prec, pitch;
    long long buf_bytes, macro_bytes;
    double gs0, gsk;
};
constexpr size_t kCkptCase = sizeof(CkptCase);
static_assert(kCkptCase == 48, "checkpoint case record is 48 bytes");

CkptCase ckpt_case(const lbm_ctx* c, size_t k)
{
    const auto& h = c->H[k];
    return CkptCase{h.nx, h.ny, c->prec, h.L.pitch, (long long)h.L.buf_bytes, (long long)h.L.macro_bytes,
                    c->P[k].cd.gs0, c->P[k].cd.gsk};
}

// The stochastic-rounding step counter a case starts from at init: the
// context's step count after the init (a single case restarts at t = 0).
unsigned init_tick(const lbm_ctx* c) { return unsigned(c->P.size() == 1 ? 0 : c->t); }

// Enqueues n steps in one persistent launch from buffer `parity`: a kernel
// that clears the arrival counters and the abort word, then the persistent
// kernel (no host waits; no memset, so the pair can be captured).
int enqueue_persistent(lbm_ctx* c, long long n, int parity)
{
    int rc = lbm::launch_persistent_reset(c->d_pcount, int(c->P.size()), c->d_pabort, c->stream);
    if (rc != 0) return rc;
    const lbm::PersistentSync sync{c->d_pcount, c->d_pabort, c->d_case_arrivals, c->spin_limit};
    return lbm::launch_persistent(c->prec, c->variant, c->d_P, c->d_work, int(c->work.size()), parity, int(n), sync,
                                  c->stream);
}

// Enqueues n step launches starting from buffer `parity` (no host waits).
int enqueue_steps(lbm_ctx* c, long long n, int parity)
{
    for (long long s = 0; s < n; ++s) {
        const int rc = lbm::launch_step(c->prec, c->variant, c->d_P, c->d_work, int(c->work.size()), parity,
                                        s == n - 1 ? 1 : 0, c->stream);
        if (rc != 0) return rc;
        parity ^= 1;
    }
    return 0;
}

// The graph of n steps from start parity p: captured from the launch
// sequence on first use, then reused (the kernel arguments depend only on
// n, p and the launch configuration).
lbm_status step_graph(lbm_ctx* c, long long n, bool persistent, hipGraphExec_t* out)
{
    const auto key = std::make_tuple(n, c->parity, persistent ? 1 : 0);
    auto it = c->graphs.find(key);
    if (it != c->graphs.end()) {
        *out = it->second;
        return LBM_OK;
    }
    HIP_TRY(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    const int rc = persistent ? enqueue_persistent(c, n, c->parity) : enqueue_steps(c, n, c->parity);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (rc != 0 || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return hip_fail(c, rc != 0 ? hipError_t(rc) : e, "step graph capture");
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t ei = hipGraphInstantiate(&exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return hip_fail(c, ei, "step graph instantiate");
    c->graphs[key] = exec;
    *out = exec;
    return LBM_OK;
}

lbm_status run_steps(lbm_ctx* c, long long n, hipEvent_t e0, hipEvent_t e1, bool graph = false,
                     bool persistent = false)
{
    for (size_t k = 0; k < c->H.size(); ++k)
        if (!c->H[k].inited) return fail(c, LBM_ESTATE, "lbm_step before lbm_init of every case");
    if (n < 0) return fail(c, LBM_EINVAL, "negative step count");
    if (persistent && !c->persistent_ok) return fail(c, LBM_EINVAL, "persistent stepping: " + c->persistent_why);
    if (persistent && n > 0x7fffffffLL) return fail(c, LBM_EINVAL, "persistent stepping: too many steps in one call");
    hipGraphExec_t exec = nullptr;
    if (graph && n > 0) {
        lbm_status st = step_graph(c, n, persistent, &exec);
        if (st != LBM_OK) return st;
    }
    if (e0) HIP_TRY(c, hipEventRecord(e0, c->stream));
    if (exec) {
        HIP_TRY(c, hipGraphLaunch(exec, c->stream));
    } else if (n > 0) {
        const int rc = persistent ? enqueue_persistent(c, n, c->parity) : enqueue_steps(c, n, c->parity);
        if (rc != 0) return hip_fail(c, hipError_t(rc), "step launch");
    }
    if (persistent && n > 0) {
        int aborted = 0;
        HIP_TRY(c, hipMemcpyAsync(&aborted, c->d_pabort, sizeof(int), hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(c, hipStreamSynchronize(c->stream));
        if (aborted) {
            for (auto& h : c->H) h.inited = false;
            return fail(c, LBM_EDEVICE, "persistent stepping: a step barrier wait gave up (spin limit); the state is "
                                        "incomplete and every case must be initialised or loaded again");
        }
    }
    c->parity ^= int(n & 1);
    if (e1) HIP_TRY(c, hipEventRecord(e1, c->stream));
    const long long t0 = c->t;
    c->t += n;
    std::vector<int> flags;
    lbm_status st = read_flags(c, flags);
    if (st != LBM_OK) return st;
    for (size_t k = 0; k < flags.size(); ++k)
        if (flags[k]) {
            if (c->H[k].diverged_at < 0) c->H[k].diverged_at = c->t;
            return fail(c, LBM_EDIVERGED, "case " + std::to_string(k) + " diverged (first seen after the step call " +
                                              "that ended at t = " + std::to_string(c->H[k].diverged_at) +
                                              "; this call covered t = " + std::to_string(t0) + " .. " +
                                              std::to_string(c->t) + ")");
        }
    return LBM_OK;
}

// ---- autotuner -------------------------------------------------------------
constexpr double kTuneMargin = 0.99;
struct TuneEntry {
    int variant = 0;
    double xw_scale = 1.0;
    int bands = 4;
    double ms = 0.0, ms_default = 0.0;
};

unsigned long long fnv1a(unsigned long long h, long long v)
{
    for (int b = 0; b < 8; ++b) {
        h ^= (unsigned long long)((v >> (8 * b)) & 0xff);
        h *= 1099511628211ULL;
    }
    return h;
}

// Cache key: device architecture, storage format and the shape signature of
// the cases (grid, walls), which is all the launch configuration depends on.
std::string tune_key(const lbm_ctx* c)
{
    static const char* prec_name[4] = {"f64", "f32", "f16s", "f32g16"};
    hipDeviceProp_t prop;
    std::string arch = "gpu";
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) {
        arch = prop.gcnArchName;
        const size_t colon = arch.find(':');
        if (colon != std::string::npos) arch = arch.substr(0, colon);
    }
    std::string key = arch + "|" + prec_name[c->prec & 3] + "|n" + std::to_string(c->P.size()) + "|";
    if (c->P.size() == 1) {
        const auto& P = c->P[0];
        key += std::to_string(P.nx) + "x" + std::to_string(P.ny) + "|w" + std::to_string(P.wall_x) +
               std::to_string(P.wall_y);
    } else {
        unsigned long long h = 1469598103934665603ULL;
        long long nodes = 0;
        for (const auto& P : c->P) {
            h = fnv1a(h, P.nx);
            h = fnv1a(h, P.ny);
            h = fnv1a(h, P.wall_x * 2 + P.wall_y);
            nodes += (long long)P.nx * P.ny;
        }
        char hex[24];
        std::snprintf(hex, sizeof hex, "%016llx", h);
        key += "nodes" + std::to_string(nodes) + "|h" + hex;
    }
    if (c->seg_rows > 0) key += "|seg" + std::to_string(c->seg_rows);
    return key;
}

double json_number(const std::string& line, const char* name, double dflt)
{
    const std::string pat = std::string("\"") + name + "\":";
    const size_t at = line.find(pat);
    if (at == std::string::npos) return dflt;
    return std::strtod(line.c_str() + at + pat.size(), nullptr);
}

// The cache file is the JSON object this library writes: one entry per line,
// "key": {"variant": v, "xw_scale": x, "bands_per_xcd": b, "ms_per_step": t,
// "default_ms_per_step": t0}.
std::map<std::string, TuneEntry> read_tune_cache(const char* path)
{
    std::map<std::string, TuneEntry> m;
    FILE* f = path ? std::fopen(path, "r") : nullptr;
    if (!f) return m;
    char buf[1024];
    while (std::fgets(buf, sizeof buf, f)) {
        const std::string line(buf);
        const size_t q0 = line.find('"');
        if (q0 == std::string::npos || line.find("\"variant\":") == std::string::npos) continue;
        const size_t q1 = line.find('"', q0 + 1);
        if (q1 == std::string::npos) continue;
        TuneEntry e;
        e.variant = int(json_number(line, "variant", 0));
        e.xw_scale = json_number(line, "xw_scale", 1.0);
        e.bands = int(json_number(line, "bands_per_xcd", 4));
        e.ms = json_number(line, "ms_per_step", 0.0);
        e.ms_default = json_number(line, "default_ms_per_step", 0.0);
        m[line.substr(q0 + 1, q1 - q0 - 1)] = e;
    }
    std::fclose(f);
    return m;
}

bool write_tune_cache(const char* path, const std::map<std::string, TuneEntry>& m)
{
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "w");
    if (!f) return false;
    std::fprintf(f, "{\n");
    size_t i = 0;
    for (const auto& kv : m) {
        const TuneEntry& e = kv.second;
        std::fprintf(f,
                     "  \"%s\": {\"variant\": %d, \"xw_scale\": %.3f, \"bands_per_xcd\": %d, "
                     "\"ms_per_step\": %.6f, \"default_ms_per_step\": %.6f}%s\n",
                     kv.first.c_str(), e.variant, e.xw_scale, e.bands, e.ms, e.ms_default, ++i < m.size() ? "," : "");
    }
    std::fprintf(f, "}\n");
    const bool ok = std::fclose(f) == 0;
    return ok && std::rename(tmp.c_str(), path) == 0;
}

}  // namespace

// ---- staging scratch of the allocation-free initialisation ---------------
// lbm_case_init stages the four host fields in a device buffer it allocates
// per call.  lbm_case_init_static stages them in this file-scope array
// instead: one copy per GPU, held until the process ends.  Host code must
// not pass the array's name to a kernel or a copy (on the host it is only a
// stand-in); it uses the device address that hipGetSymbolAddress returns,
// looked up once per device with that device current.
constexpr long long kInitScratchNodes = 1LL << 20;   // 4 fields x 2^20 doubles = 32 MiB
static __device__ __align__(256) double scratch[4 * kInitScratchNodes];

__global__ void fill_doubles(double* __restrict__ p, long long n, double v)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}

__global__ void clear_flag(int* flag) { *flag = 0; }
__global__ void set_word(unsigned* p, unsigned v) { *p = v; }

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the context's device (looked up on first use
// there, with that device current).
lbm_status scratch_on_device(lbm_ctx* c, double** out)
{
    if (c->device < 0 || c->device >= kMaxDevices) return fail(c, LBM_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[c->device]) {
        int prev = 0;
        HIP_TRY(c, hipGetDevice(&prev));
        if (prev != c->device) HIP_TRY(c, hipSetDevice(c->device));
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (prev != c->device) (void)hipSetDevice(prev);
        if (e != hipSuccess) return hip_fail(c, e, "hipGetSymbolAddress(scratch)");
        if (!p) return fail(c, LBM_EDEVICE, "hipGetSymbolAddress(scratch) returned no address");
        g_scratch[c->device] = static_cast<double*>(p);
    }
    *out = g_scratch[c->device];
    return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm_workspace_bytes(int nx, int ny, int prec)
{
    if (nx < 1 || ny < 1 || prec < 0 || prec > 3) return 0;
    return layout_of(nx, ny, prec).total;
}

lbm_status lbm_create(int nx, int ny, const lbm_eos* eos, double Pr, double gamma, const lbm_relax* relax,
                      const lbm_boundary* bc, const lbm_options* opt, lbm_ctx** out)
{
    return create_impl(1, &nx, &ny, eos, &Pr, &gamma, relax, bc, opt, nullptr, 0, out);
}

lbm_status lbm_create_ex(int nx, int ny, const lbm_eos* eos, double Pr, double gamma, const lbm_relax* relax,
                         const lbm_boundary* bc, const lbm_options* opt, void* dev_workspace, size_t bytes,
                         lbm_ctx** out)
{
    if (!dev_workspace) {
        if (out) *out = nullptr;
        return LBM_EINVAL;
    }
    return create_impl(1, &nx, &ny, eos, &Pr, &gamma, relax, bc, opt, dev_workspace, bytes, out);
}

lbm_status lbm_batch_create(int ncases, const int* nx, const int* ny, const lbm_eos* eos, const double* Pr,
                            const double* gamma, const lbm_relax* relax, const lbm_boundary* bc,
                            const lbm_options* opt, lbm_ctx** out)
{
    if (!nx || !ny || !eos || !Pr || !gamma || !relax || !bc || !opt) {
        if (out) *out = nullptr;
        return LBM_EINVAL;
    }
    return create_impl(ncases, nx, ny, eos, Pr, gamma, relax, bc, opt, nullptr, 0, out);
}

int lbm_batch_size(const lbm_ctx* c) { return c ? int(c->P.size()) : 0; }

long long lbm_work_items(const lbm_ctx* c) { return c ? c->n_items : 0; }

lbm_status lbm_case_init(lbm_ctx* c, int k, const double* rho, const double* ux, const double* uy, const double* T)
{
    lbm_status st = check_case(c, k);
    if (st != LBM_OK) return st;
    const auto& P = c->P[k];
    const size_t nn = size_t(P.nx) * P.ny;
    std::vector<double> h(4 * nn);
    for (size_t i = 0; i < nn; ++i) {
        h[i] = rho ? rho[i] : P.cd.rho0;
        h[nn + i] = ux ? ux[i] : 0.0;
        h[2 * nn + i] = uy ? uy[i] : 0.0;
        h[3 * nn + i] = T ? T[i] : P.cd.T0;
        if (!(h[i] > 0) || !(h[3 * nn + i] > 0) || !std::isfinite(h[i]) || !std::isfinite(h[nn + i]) ||
            !std::isfinite(h[2 * nn + i]) || !std::isfinite(h[3 * nn + i]))
            return fail(c, LBM_EINVAL, "initial fields must be finite with rho > 0 and T > 0");
    }
    void* d = nullptr;
    HIP_TRY(c, hipMalloc(&d, h.size() * sizeof(double)));
    hipError_t e = hipMemcpyAsync(d, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, c->stream);
    if (e == hipSuccess) e = hipMemsetAsync(P.flag, 0, sizeof(int), c->stream);
    int rc = 0;
    if (e == hipSuccess)
        rc = lbm::launch_init(c->prec, c->d_P, k, (long long)nn, static_cast<const double*>(d), c->parity,
                              init_tick(c), c->stream);
    if (e == hipSuccess && rc == 0) e = hipStreamSynchronize(c->stream);
    (void)hipFree(d);
    if (e != hipSuccess) return hip_fail(c, e, "lbm_init");
    if (rc != 0) return hip_fail(c, hipError_t(rc), "init launch");
    c->H[k].inited = true;
    c->H[k].diverged_at = -1;
    if (c->P.size() == 1) c->t = 0;
    return LBM_OK;
}

lbm_status lbm_init(lbm_ctx* c, const double* rho, const double* ux, const double* uy, const double* T)
{
    return lbm_case_init(c, 0, rho, ux, uy, T);
}

lbm_status lbm_case_init_static(lbm_ctx* c, int k, const double* rho, const double* ux, const double* uy,
                                const double* T)
{
    lbm_status st = check_case(c, k);
    if (st != LBM_OK) return st;
    const auto& P = c->P[k];
    const long long nn = (long long)P.nx * P.ny;
    if (nn > kInitScratchNodes)
        return fail(c, LBM_EINVAL, "grid of " + std::to_string(nn) + " nodes exceeds the static init scratch (" +
                                       std::to_string(kInitScratchNodes) + " nodes); use lbm_case_init");
    const double* src[4] = {rho, ux, uy, T};
    for (long long i = 0; i < nn; ++i) {
        const double r = rho ? rho[i] : P.cd.rho0, t = T ? T[i] : P.cd.T0;
        if (!(r > 0) || !(t > 0) || !std::isfinite(r) || !std::isfinite(t) || (ux && !std::isfinite(ux[i])) ||
            (uy && !std::isfinite(uy[i])))
            return fail(c, LBM_EINVAL, "initial fields must be finite with rho > 0 and T > 0");
    }
    double* d = nullptr;
    st = scratch_on_device(c, &d);
    if (st != LBM_OK) return st;
    const double dflt[4] = {P.cd.rho0, 0.0, 0.0, P.cd.T0};
    for (int f = 0; f < 4; ++f) {
        if (src[f]) {
            HIP_TRY(c, hipMemcpyAsync(d + f * nn, src[f], size_t(nn) * sizeof(double), hipMemcpyHostToDevice, c->stream));
        } else {
            hipLaunchKernelGGL(fill_doubles, dim3(unsigned(std::min<long long>((nn + 255) / 256, 4096))), dim3(256), 0,
                               c->stream, d + f * nn, nn, dflt[f]);
            HIP_TRY(c, hipGetLastError());
        }
    }
    hipLaunchKernelGGL(clear_flag, dim3(1), dim3(1), 0, c->stream, P.flag);
    HIP_TRY(c, hipGetLastError());
    const int rc = lbm::launch_init(c->prec, c->d_P, k, nn, d, c->parity, init_tick(c), c->stream);
    if (rc != 0) return hip_fail(c, hipError_t(rc), "init launch");
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->H[k].inited = true;
    if (c->P.size() == 1) c->t = 0;
    return LBM_OK;
}

lbm_status lbm_step(lbm_ctx* c, long long n)
{
    lbm_status st = check_ctx(c);
    if (st != LBM_OK) return st;
    return run_steps(c, n, nullptr, nullptr);
}

lbm_status lbm_step_timed(lbm_ctx* c, long long n, double* ms)
{
    lbm_status st = check_ctx(c);
    if (st != LBM_OK) return st;
    hipEvent_t e0, e1;
    HIP_TRY(c, hipEventCreate(&e0));
    HIP_TRY(c, hipEventCreate(&e1));
    st = run_steps(c, n, e0, e1);
    if (st == LBM_OK || st == LBM_EDIVERGED) {
        float f = 0.f;
        if (hipEventElapsedTime(&f, e0, e1) == hipSuccess && ms) *ms = f;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return st;
}

lbm_status lbm_step_ex(lbm_ctx* c, long long n, int flags, double* ms)
{
    lbm_status st = check_ctx(c);
    if (st != LBM_OK) return st;
    if (flags & ~(LBM_STEP_GRAPH | LBM_STEP_PERSISTENT)) return fail(c, LBM_EINVAL, "unknown step flags");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (ms) {
        HIP_TRY(c, hipEventCreate(&e0));
        HIP_TRY(c, hipEventCreate(&e1));
    }
    st = run_steps(c, n, e0, e1, (flags & LBM_STEP_GRAPH) != 0, (flags & LBM_STEP_PERSISTENT) != 0);
    if (ms && (st == LBM_OK || st == LBM_EDIVERGED)) {
        float f = 0.f;
        if (hipEventElapsedTime(&f, e0, e1) == hipSuccess) *ms = f;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    return st;
}

lbm_status lbm_set_persistent_spin_limit(lbm_ctx* c, unsigned polls)
{
    lbm_status st = check_ctx(c);
    if (st != LBM_OK) return st;
    c->spin_limit = polls;
    drop_graphs(c);
    return LBM_OK;
}

long long lbm_case_diverged_at(const lbm_ctx* c, int k)
{
    if (!c || k < 0 || k >= int(c->H.size())) return -1;
    return c->H[k].diverged_at;
}

lbm_status lbm_set_launch_config(lbm_ctx* c, int variant, double xw_scale, int bands_per_xcd)
{
    lbm_status st = check_ctx(c);
    if (st != LBM_OK) return st;
    return configure(c, variant, xw_scale, bands_per_xcd);
}

lbm_status lbm_autotune(lbm_ctx* c, int trial_steps, const char* cache_path, lbm_tune_result* out)
{
    lbm_status st = check_ctx(c);
    if (st != LBM_OK) return st;
    for (const auto& h : c->H)
        if (!h.inited) return fail(c, LBM_ESTATE, "lbm_autotune before lbm_init of every case");
    if (trial_steps < 0) return fail(c, LBM_EINVAL, "negative trial step count");
    const std::string key = tune_key(c);
    std::map<std::string, TuneEntry> cache = read_tune_cache(cache_path);
    auto hit = cache.find(key);
    if (hit != cache.end()) {
        const TuneEntry& e = hit->second;
        st = configure(c, e.variant, e.xw_scale, e.bands);
        if (st != LBM_OK) return st;
        if (out) *out = lbm_tune_result{e.variant, e.xw_scale, e.bands, e.ms, e.ms_default, 0, 1};
        return LBM_OK;
    }
    long long nodes = 0;
    bool xwall = false;
    for (const auto& P : c->P) {
        nodes += (long long)P.nx * P.ny;
        xwall = xwall || P.wall_x;
    }
    if (trial_steps == 0) trial_steps = int(std::min<long long>(200, std::max<long long>(5, 20000000LL / std::max(nodes, 1LL))));
    // the trials advance the state: keep the current buffer, macros and flag
    // of every case and put them back after each trial
    size_t bytes = 0;
    for (const auto& h : c->H) bytes += h.L.buf_bytes + h.L.macro_bytes + h.L.flag_bytes;
    void* backup = nullptr;
    if (hipMalloc(&backup, bytes) != hipSuccess) return fail(c, LBM_ENOMEM, "hipMalloc of the tuner's state copy failed");
    const int parity0 = c->parity;
    const long long t0 = c->t;
    auto copy_state = [&](bool save) -> hipError_t {
        char* b = static_cast<char*>(backup);
        for (const auto& h : c->H) {
            char* cur = h.base + parity0 * h.L.buf_bytes;
            char* rest = h.base + 2 * h.L.buf_bytes;   // macros, then the flag
            const size_t rb = h.L.macro_bytes + h.L.flag_bytes;
            hipError_t e = hipMemcpyAsync(save ? b : cur, save ? cur : b, h.L.buf_bytes, hipMemcpyDeviceToDevice, c->stream);
            if (e != hipSuccess) return e;
            b += h.L.buf_bytes;
            e = hipMemcpyAsync(save ? b : rest, save ? rest : b, rb, hipMemcpyDeviceToDevice, c->stream);
            if (e != hipSuccess) return e;
            b += rb;
        }
        return hipStreamSynchronize(c->stream);
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t he = copy_state(true);
    if (he == hipSuccess) he = hipEventCreate(&e0);
    if (he == hipSuccess) he = hipEventCreate(&e1);
    const int v0 = c->variant;
    const double x0 = c->xw_scale;
    const int b0 = c->bands_per_xcd;
    TuneEntry best, dflt;
    best.ms = 1e300;
    int trials = 0;
    const double scales[3] = {1.0, 0.85, 1.2};
    const int bands[4] = {4, 1, 8, 16};
    for (int v = 0; v < lbm::NUM_STEP_VARIANTS && he == hipSuccess && st == LBM_OK; ++v)
        for (int si = 0; si < (xwall ? 3 : 1) && he == hipSuccess && st == LBM_OK; ++si)
            for (int bi = 0; bi < 4 && he == hipSuccess && st == LBM_OK; ++bi) {
                st = configure(c, v, scales[si], bands[bi]);
                if (st != LBM_OK) break;
                double ms_best = 1e300;
                for (int rep = 0; rep < 4; ++rep) {   // the first run warms up
                    he = copy_state(false);
                    if (he != hipSuccess) break;
                    c->parity = parity0;
                    const lbm_status rs = run_steps(c, trial_steps, e0, e1);
                    if (rs != LBM_OK && rs != LBM_EDIVERGED) {
                        st = rs;
                        break;
                    }
                    float f = 0.f;
                    he = hipEventElapsedTime(&f, e0, e1);
                    if (he != hipSuccess) break;
                    if (rep > 0) ms_best = std::min(ms_best, double(f) / trial_steps);
                }
                ++trials;
                if (v == 0 && si == 0 && bi == 0) dflt.ms = ms_best;
                if (ms_best < best.ms) {
                    best.variant = v;
                    best.xw_scale = scales[si];
                    best.bands = bands[bi];
                    best.ms = ms_best;
                }
            }
    if (he == hipSuccess) he = copy_state(false);
    c->parity = parity0;
    c->t = t0;
    for (auto& h : c->H) h.diverged_at = -1;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(backup);
    if (st == LBM_OK && he != hipSuccess) st = hip_fail(c, he, "autotune trial");
    if (st != LBM_OK) {
        (void)configure(c, v0, x0, b0);
        return st;
    }
    best.ms_default = dflt.ms;
    // keep the hand-tuned default unless a configuration beats it by more
    // than the trial-to-trial spread of short timings (1 %)
    if (!(best.ms < kTuneMargin * dflt.ms)) {
        best.variant = 0;
        best.xw_scale = 1.0;
        best.bands = 4;
        best.ms = dflt.ms;
    }
    st = configure(c, best.variant, best.xw_scale, best.bands);
    if (st != LBM_OK) return st;
    if (cache_path) {
        cache[key] = best;
        if (!write_tune_cache(cache_path, cache)) return fail(c, LBM_EINVAL, "cannot write the tuning cache file");
    }
    if (out) *out = lbm_tune_result{best.variant, best.xw_scale, best.bands, best.ms, best.ms_default, trials, 0};
    return LBM_OK;
}

lbm_status lbm_case_macros(lbm_ctx* c, int k, double* rho, double* ux, double* uy, double* T, double* p)
{
    lbm_status st = check_case(c, k);
    if (st != LBM_OK) return st;
    if (!c->H[k].inited) return fail(c, LBM_ESTATE, "case not initialised");
    const auto& P = c->P[k];
    const size_t nn = size_t(P.nx) * P.ny;
    double* outs[5] = {rho, ux, uy, T, p};
    for (int f = 0; f < 5; ++f)
        if (outs[f])
            HIP_TRY(c, hipMemcpyAsync(outs[f], P.macro + f * nn, nn * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status lbm_macros(lbm_ctx* c, double* rho, double* ux, double* uy, double* T, double* p)
{
    return lbm_case_macros(c, 0, rho, ux, uy, T, p);
}

lbm_status lbm_case_nusselt(lbm_ctx* c, int k, int side, double* nu)
{
    lbm_status st = check_case(c, k);
    if (st != LBM_OK) return st;
    if (!c->H[k].inited) return fail(c, LBM_ESTATE, "case not initialised");
    const auto& P = c->P[k];
    if (side < 0 || side > 3 || !nu) return fail(c, LBM_EINVAL, "bad side");
    const int lo = side < 2 ? 0 : 2;
    const bool walled = side < 2 ? P.wall_x : P.wall_y;
    if (!walled || P.side_adiabatic[lo] || P.side_adiabatic[lo + 1] || P.cd.side_T[lo] == P.cd.side_T[lo + 1])
        return fail(c, LBM_EINVAL, "Nusselt number needs Dirichlet walls with a temperature difference");
    const int rc = lbm::launch_nusselt(c->d_P, k, side, c->d_red, c->stream);
    if (rc != 0) return hip_fail(c, hipError_t(rc), "nusselt launch");
    HIP_TRY(c, hipMemcpyAsync(nu, c->d_red, sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status lbm_nusselt(lbm_ctx* c, int side, double* nu) { return lbm_case_nusselt(c, 0, side, nu); }

lbm_status lbm_case_totals(lbm_ctx* c, int k, double* mass, double* momx, double* momy, double* energy)
{
    lbm_status st = check_case(c, k);
    if (st != LBM_OK) return st;
    if (!c->H[k].inited) return fail(c, LBM_ESTATE, "case not initialised");
    const int rc = lbm::launch_totals(c->d_P, k, c->d_red, kRedBlocks, c->d_red + kRedBlocks * 4, c->stream);
    if (rc != 0) return hip_fail(c, hipError_t(rc), "totals launch");
    double h[4];
    HIP_TRY(c, hipMemcpyAsync(h, c->d_red + kRedBlocks * 4, sizeof h, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    if (mass) *mass = h[0];
    if (momx) *momx = h[1];
    if (momy) *momy = h[2];
    if (energy) *energy = h[3];
    return LBM_OK;
}

lbm_status lbm_totals(lbm_ctx* c, double* mass, double* momx, double* momy, double* energy)
{
    return lbm_case_totals(c, 0, mass, momx, momy, energy);
}

lbm_status lbm_batch_flags(lbm_ctx* c, int* diverged)
{
    lbm_status st = check_ctx(c);
    if (st != LBM_OK) return st;
    if (!diverged) return fail(c, LBM_EINVAL, "null output");
    std::vector<int> flags;
    st = read_flags(c, flags);
    if (st != LBM_OK) return st;
    for (size_t k = 0; k < flags.size(); ++k) diverged[k] = flags[k] ? 1 : 0;
    return LBM_OK;
}

lbm_status lbm_batch_step(lbm_ctx* c, long long n)
{
    lbm_status st = check_ctx(c);
    if (st != LBM_OK) return st;
    st = run_steps(c, n, nullptr, nullptr);
    return st == LBM_EDIVERGED ? LBM_OK : st;   // per-case flags are reported by lbm_batch_nusselt
}

lbm_status lbm_batch_nusselt(lbm_ctx* c, int side, double* nu, int* diverged)
{
    lbm_status st = check_ctx(c);
    if (st != LBM_OK) return st;
    if (!nu || !diverged) return fail(c, LBM_EINVAL, "null output");
    if (side < 0 || side > 3) return fail(c, LBM_EINVAL, "bad side");
    std::vector<int> flags;
    st = read_flags(c, flags);
    if (st != LBM_OK) return st;
    for (size_t k = 0; k < c->P.size(); ++k) {
        const auto& P = c->P[k];
        const int lo = side < 2 ? 0 : 2;
        const bool walled = side < 2 ? P.wall_x : P.wall_y;
        const bool pair = walled && !P.side_adiabatic[lo] && !P.side_adiabatic[lo + 1] &&
                          P.cd.side_T[lo] != P.cd.side_T[lo + 1];
        diverged[k] = flags[k] ? 1 : 0;
        nu[k] = NAN;
        if (flags[k] || !pair || !c->H[k].inited) continue;
        st = lbm_case_nusselt(c, int(k), side, &nu[k]);
        if (st != LBM_OK) return st;
    }
    return LBM_OK;
}

size_t lbm_state_bytes(const lbm_ctx* c)
{
    if (!c) return 0;
    size_t s = kCkptHeader + c->H.size() * kCkptCase;
    for (const auto& h : c->H) s += h.L.buf_bytes + h.L.macro_bytes;
    return s;
}

lbm_status lbm_save(lbm_ctx* c, void* host, size_t bytes)
{
    lbm_status st = check_ctx(c);
    if (st != LBM_OK) return st;
    if (!host || bytes < lbm_state_bytes(c)) return fail(c, LBM_EINVAL, "buffer smaller than lbm_state_bytes");
    char* o = static_cast<char*>(host);
    const long long hdr[2] = {c->t, (long long)c->P.size()};
    std::memcpy(o, kCkptMagic, 8);
    std::memcpy(o + 8, hdr, 16);
    o += kCkptHeader;
    for (size_t k = 0; k < c->H.size(); ++k) {
        const CkptCase cc = ckpt_case(c, k);
        std::memcpy(o, &cc, kCkptCase);
        o += kCkptCase;
    }
    for (size_t k = 0; k < c->H.size(); ++k) {
        const auto& h = c->H[k];
        HIP_TRY(c, hipMemcpyAsync(o, h.base + c->parity * h.L.buf_bytes, h.L.buf_bytes, hipMemcpyDeviceToHost, c->stream));
        o += h.L.buf_bytes;
        HIP_TRY(c, hipMemcpyAsync(o, h.base + 2 * h.L.buf_bytes, h.L.macro_bytes, hipMemcpyDeviceToHost, c->stream));
        o += h.L.macro_bytes;
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    return LBM_OK;
}

lbm_status lbm_load(lbm_ctx* c, const void* host, size_t bytes)
{
    lbm_status st = check_ctx(c);
    if (st != LBM_OK) return st;
    if (!host || bytes < kCkptHeader) return fail(c, LBM_EINVAL, "buffer smaller than a checkpoint header");
    const char* o = static_cast<const char*>(host);
    if (std::memcmp(o, kCkptMagic, 8) != 0) return fail(c, LBM_EINVAL, "not a checkpoint of this library (format tag)");
    long long hdr[2];
    std::memcpy(hdr, o + 8, 16);
    if (hdr[1] != (long long)c->P.size()) return fail(c, LBM_EINVAL, "checkpoint has a different number of cases");
    if (bytes < lbm_state_bytes(c)) return fail(c, LBM_EINVAL, "buffer smaller than lbm_state_bytes");
    o += kCkptHeader;
    for (size_t k = 0; k < c->H.size(); ++k) {
        CkptCase cc;
        std::memcpy(&cc, o, kCkptCase);
        o += kCkptCase;
        const CkptCase mine = ckpt_case(c, k);
        if (std::memcmp(&cc, &mine, kCkptCase) != 0)
            return fail(c, LBM_EINVAL, "checkpoint case " + std::to_string(k) +
                                           " differs in grid, precision or layout from this context");
    }
    for (size_t k = 0; k < c->H.size(); ++k) {
        auto& h = c->H[k];
        HIP_TRY(c, hipMemcpyAsync(h.base + c->parity * h.L.buf_bytes, o, h.L.buf_bytes, hipMemcpyHostToDevice, c->stream));
        o += h.L.buf_bytes;
        HIP_TRY(c, hipMemcpyAsync(h.base + 2 * h.L.buf_bytes, o, h.L.macro_bytes, hipMemcpyHostToDevice, c->stream));
        o += h.L.macro_bytes;
        HIP_TRY(c, hipMemsetAsync(c->P[k].flag, 0, sizeof(int), c->stream));
        hipLaunchKernelGGL(set_word, dim3(1), dim3(1), 0, c->stream, c->P[k].tick + c->parity, unsigned(hdr[0]));
        HIP_TRY(c, hipGetLastError());
        h.inited = true;
        h.diverged_at = -1;
    }
    HIP_TRY(c, hipStreamSynchronize(c->stream));
    c->t = hdr[0];
    return LBM_OK;
}

long long lbm_time(const lbm_ctx* c) { return c ? c->t : 0; }

lbm_status lbm_copy_bandwidth(size_t bytes, int iters, void* hip_stream, double* gbps, double* ms_per_copy)
{
    if (bytes < 16 || bytes % 16 || iters < 1) return LBM_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    void *a = nullptr, *b = nullptr;
    if (hipMalloc(&a, bytes) != hipSuccess) return LBM_ENOMEM;
    if (hipMalloc(&b, bytes) != hipSuccess) {
        (void)hipFree(a);
        return LBM_ENOMEM;
    }
    lbm_status rc = LBM_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    float ms = 0.f;
    if (hipMemsetAsync(a, 0, bytes, st) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
        hipEventCreate(&e1) != hipSuccess) {
        rc = LBM_EDEVICE;
    } else {
        lbm::launch_copy(a, b, (long long)bytes, st);   // warm-up
        (void)hipEventRecord(e0, st);
        for (int i = 0; i < iters; ++i) lbm::launch_copy(a, b, (long long)bytes, st);
        (void)hipEventRecord(e1, st);
        if (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) rc = LBM_EDEVICE;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipFree(a);
    (void)hipFree(b);
    if (rc == LBM_OK) {
        const double per = ms / iters;
        if (ms_per_copy) *ms_per_copy = per;
        if (gbps) *gbps = 2.0 * double(bytes) / (per * 1e-3) / 1e9;
    }
    return rc;
}

const char* lbm_last_error(const lbm_ctx* c) { return c ? c->err.c_str() : "null context"; }

void lbm_destroy(lbm_ctx* c)
{
    if (!c) return;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    drop_graphs(c);
    if (c->d_work) (void)hipFree(c->d_work);
    if (c->d_case_arrivals) (void)hipFree(c->d_case_arrivals);
    if (c->d_pcount) (void)hipFree(c->d_pcount);
    if (c->d_pabort) (void)hipFree(c->d_pabort);
    for (void* p : c->allocs) (void)hipFree(p);
    if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

}  // extern "C"

unsigned lbm_rounding_operand(int prec, int x, int y, unsigned t, int q)
{
    if (q < 0 || q > 17) return 0u;
    if (prec == LBM_FP16S) return lbm::sr::operand_at(x, y, t, q);
    if (prec == LBM_F32G16 && q >= 9) return lbm::sr::operand_at(x, y, t, q - 9);
    return 0u;
}

double lbm_round_half_stochastic(float v, unsigned r) { return lbm::round_half_stochastic_model(v, r); }

lbm_status lbm_round_half_device(const float* v, const unsigned* r, float* out, long long n, void* hip_stream)
{
    if (n < 0 || (n > 0 && (!v || !r || !out))) return LBM_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    const int rc = lbm::launch_round_half(v, r, out, n, st);
    if (rc != 0) return LBM_EDEVICE;
    return hipStreamSynchronize(st) == hipSuccess ? LBM_OK : LBM_EDEVICE;
}
