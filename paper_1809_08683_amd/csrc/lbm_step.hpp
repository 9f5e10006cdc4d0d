// Step and initialisation kernels of the coupled D2Q9 MRT scheme (Huang, Wu &
// Adams, arXiv:1809.08683) for gfx950, as templates over the storage format
// and its tuning variant.  Each storage format is instantiated in a
// translation unit of its own (lbm_step_<format>.hip), so that the formats
// compile in parallel.
//
// Storage: two ping-pong buffers of (ny + 2) stored row blocks; a row block
// holds 18 rows of `pitch` elements, one per DF (f_0..f_8, g_0..g_8), so DF q
// of node (x, y) sits at element ((y + 1) * 18 + q) * pitch + slot(x).  Along
// a DF row the columns are kept in 64-slot strip regions (see CaseParams):
// each interior wavefront stores the 62 own slots of its region; its edge
// lanes pull the neighbouring strips' edge columns from their regions.  The extra
// stored rows, and slots 0-1 of the first region and the two slots after the
// last column on walled sides, hold ghost cells: a wall node writes every
// post-collision DF that would leave the domain into the ghost cell it would
// reach, in the row of the opposite direction, so the next step's pull reads
// the bounce-back temporaries of eqs. BB.f and BB.g without any special case.
// Periodic sides wrap in the index arithmetic.
//
// One step is one launch.  Each wavefront takes one work item:
//   - interior item: 64 lanes span 62 output columns plus one halo column
//     on each side and march up a segment of rows with a rolling window of
//     three rows of (rho, p), so that grad(rho) and grad(p) of the correction
//     terms use same-time-level neighbours; x-neighbours come from lane
//     shuffles, y-neighbours from the window;
//   - wall item: 64 wall nodes; each lane completes its node's macros
//     (Sec. 3.1), extrapolates the tilde non-equilibrium moments from x_f,
//     x_ff (eqs. neq.redefinition, neq.extrapolation), inverts them with the
//     closed forms of App. B, collides and writes its ghost cells.
#pragma once
#include <algorithm>

#include "lbm_device.hpp"
#include "lbm_launch.hpp"

namespace lbm {

constexpr int WAVE = 64;

// Storage format of the DFs: element type of the nine f rows and of the
// nine g rows of a stored row block (both decode to the arithmetic type C).
template <typename SF, typename SG>
struct Format {
    using F = SF;
    using G = SG;
    using C = typename Store<SF>::C;
    static_assert(sizeof(typename Store<SG>::C) == sizeof(C), "f and g rows share one arithmetic type");
    static constexpr int EF = int(sizeof(SF)), EG = int(sizeof(SG));
};
using FmtF64 = Format<double, double>;
using FmtF32 = Format<float, float>;
using FmtF16 = Format<__half, __half>;
using FmtF32G16 = Format<float, __half>;

// Per storage format: the wavefronts per SIMD that the register budget of
// the step kernel allows; whether the interior waves of a block advance row
// by row together (a barrier per row, so that the edge lanes of neighbouring
// strips read the lines their neighbours fetch at the same moment); whether
// the strips next to an x-wall select the wall state of their wall lanes
// instead of branching (needs a few more registers); whether segments of a
// band alternate their march direction (the 16-bit format spills with it);
// whether the strips next to an x-wall collide its nodes (else wall items
// take them; FP64 has no registers to spare for it), the time of a row of
// such a strip relative to a plain row, and whether it loads the row two
// ahead before the collision (where the registers allow it); whether the
// moments of the row ahead wait in the wavefront's LDS slice during the
// collision; the wavefronts of a block (neighbouring strips of a segment
// share its CU); and whether a wavefront lowers its priority as it advances
// (FP64 ran 0.6 % faster without, the other formats 2-13 % slower).
template <typename Fm> struct Tuning;
template <> struct Tuning<FmtF64> {
    static constexpr int block_waves = 8;
    static constexpr bool park = true;
    static constexpr int waves = 2;
    static constexpr bool lockstep = true, edge_select = true, alternate = true;
    static constexpr bool xw_strips = false, xw_prefetch = false;
    static constexpr double xw_cost = 1.0;
    static constexpr bool fair = false;
};
template <> struct Tuning<FmtF32> {
    static constexpr int block_waves = 4;
    static constexpr bool park = true;
    static constexpr int waves = 3;
    static constexpr bool lockstep = true, edge_select = true, alternate = true;
    static constexpr bool xw_strips = true, xw_prefetch = true;
    static constexpr double xw_cost = 1.15;
    static constexpr bool fair = true;
};
template <> struct Tuning<FmtF32G16> {
    static constexpr int block_waves = 4;
    static constexpr bool park = true;
    static constexpr int waves = 3;
    static constexpr bool lockstep = true, edge_select = true, alternate = true;
    static constexpr bool xw_strips = true, xw_prefetch = true;
    static constexpr double xw_cost = 1.3;
    static constexpr bool fair = true;
};
template <> struct Tuning<FmtF16> {
    static constexpr int block_waves = 8;
    static constexpr bool park = true;
    static constexpr int waves = 4;
    static constexpr bool lockstep = false, edge_select = false, alternate = false;
    static constexpr bool xw_strips = true, xw_prefetch = false;
    static constexpr double xw_cost = 2.0;
    static constexpr bool fair = true;
};
// Tuning variants of a format, for the autotuner (lbm_autotune): variant 0
// is the hand-tuned set above; 1 flips the progress priority, 2 flips the
// LDS parking of the ahead row, 3 takes the other block size (4 <-> 8
// wavefronts), 4 flips the lockstep march.  Everything else stays that of
// the format.  The host builds the work list from the variant's shape (block
// size, lockstep, occupancy; step_shape_v), so the two always match.
template <typename Base, int V>
struct Variant : Base {
};
template <typename Base, int V>
struct Tuning<Variant<Base, V>> : Tuning<Base> {
    static constexpr bool fair = (V == 1) != Tuning<Base>::fair;
    static constexpr bool park = (V == 2) != Tuning<Base>::park;
    static constexpr int block_waves = V == 3 ? (Tuning<Base>::block_waves == 8 ? 4 : 8) : Tuning<Base>::block_waves;
    static constexpr bool lockstep = (V == 4) != Tuning<Base>::lockstep;
};
static_assert(NUM_STEP_VARIANTS == 5, "variants 0-4 are defined above");

static_assert(REGION_SLOTS == WAVE && STRIP_COLS == WAVE - 2, "one wavefront per strip region");

#define EXq(q) ((q) == 1 || (q) == 5 || (q) == 8 ? 1 : ((q) == 3 || (q) == 6 || (q) == 7 ? -1 : 0))
#define EYq(q) ((q) == 2 || (q) == 5 || (q) == 6 ? 1 : ((q) == 4 || (q) == 7 || (q) == 8 ? -1 : 0))
#define OPPq(q) ((q) == 0 ? 0 : ((q) <= 4 ? (((q) + 1) % 4) + 1 : (((q) - 5 + 2) % 4) + 5))

__device__ __forceinline__ int wrap_axis(int v, int n, int walled)
{
    if (walled) return v;
    v %= n;
    return v < 0 ? v + n : v;
}

__device__ __forceinline__ int floor_div(int a, int b) { return a >= 0 ? a / b : -((-a + b - 1) / b); }

// storage slot of column x in [-1, nx] (wrapped on a periodic axis) within a
// stored DF row: the slot of its owning strip; the left wall column is slot 0
// of strip 0, the right wall and ghost columns follow the last strip's
// columns, and the left ghost column is the row's last slot
__device__ __forceinline__ int col_slot(const CaseParams& P, int x)
{
    x = wrap_axis(x, P.nx, P.wall_x);
    if (x < 0) return P.pitch - 1;
    const int r = min(max(floor_div(x - P.xlo, STRIP_COLS), 0), P.nstrips - 1);
    return r * REGION_SLOTS + (x - P.xlo - r * STRIP_COLS) + 1;
}

// Calls fn(slot) for the slot that holds column x (the layout keeps one).
template <typename F>
__device__ __forceinline__ void for_each_slot(const CaseParams& P, int x, F&& fn)
{
    fn(col_slot(P, x));
}

// Bytes of one stored row block and the byte offset of DF row q (0..17)
// inside it: the nine f rows, then the nine g rows.
template <typename Fm>
__device__ __forceinline__ long long block_bytes(const CaseParams& P)
{
    return 9LL * P.pitch * (Fm::EF + Fm::EG);
}
template <typename Fm>
__device__ __forceinline__ long long row_offset(const CaseParams& P, int q)
{
    return q < 9 ? (long long)q * P.pitch * Fm::EF : 9LL * P.pitch * Fm::EF + (long long)(q - 9) * P.pitch * Fm::EG;
}

// byte offset of DF row q of lattice row y in [-1, ny] (stored row y + 1)
template <typename Fm>
__device__ __forceinline__ long long row_byte(const CaseParams& P, int q, int y)
{
    return (long long)(wrap_axis(y, P.ny, P.wall_y) + 1) * block_bytes<Fm>(P) + row_offset<Fm>(P, q);
}

template <typename Fm> __device__ __forceinline__ typename Fm::C load_df(const char* buf, int q, long long off)
{
    using F = typename Fm::F;
    using G = typename Fm::G;
    return q < 9 ? Store<F>::load(reinterpret_cast<const F*>(buf + off)) : Store<G>::load(reinterpret_cast<const G*>(buf + off));
}
// store of DF row q (0..17) with the random operand rnd of its stochastic rounding
template <typename Fm> __device__ __forceinline__ void store_df(char* buf, int q, long long off, typename Fm::C v,
                                                                unsigned rnd)
{
    using F = typename Fm::F;
    using G = typename Fm::G;
    if (q < 9) Store<F>::store_sr(reinterpret_cast<F*>(buf + off), v, rnd);
    else Store<G>::store_sr(reinterpret_cast<G*>(buf + off), v, rnd);
}
template <typename Fm> __device__ __forceinline__ long long slot_bytes(int q, int slot)
{
    return (long long)slot * (q < 9 ? Fm::EF : Fm::EG);
}

// Reference of the 16-bit g rows (FP32 f + FP16 g and FP16S storage).  In a cavity
// between Dirichlet x-walls the rest deviation g - g_rest is O(Delta T)
// everywhere, and the FP16 rounding of it limits the heat flux at the walls.
// The g rows of that format therefore store g - g_ref(x), where g_ref is the
// rest equilibrium of the conduction state: T_ref linear between the wall
// temperatures and rho_ref T_ref = rho0 T0 (uniform ideal-gas pressure).  At
// rest, n^eq (Sec. 2.2) depends on the state only through rho E, which is
// uniform there, and rho0 C_p T in rows 1 and 2, so
//   g_ref - g_rest = M^-1 (0, 4 + gamma1, -4 + gamma2, 0, ..., 0) s(x),
//   s(x) = rho0 C_p (T_ref(x) - T0) = gs0 + gsk x,
// an offset v_q s(x) per DF that costs no stored bytes.  Every store of a g
// row subtracts the offset of the column it is stored in and every load adds
// it back, so the reference never changes what the scheme computes, only
// what the 16-bit rows round.  The interior march applies it to the moments
// instead: a pull reads DF q from column x - e_qx, and
//   M [v_q s(x - e_qx)]_q = s(x) (0, 4 + gamma1, -4 + gamma2, 0, ...)
//                           - gsk (0, 0, 0, sum_q e_qx^2 v_q, sum_q M_4q e_qx v_q, 0, ...).
namespace gref {
constexpr double a1 = (4.0 + mc::gamma1) / 36.0, a2 = (-4.0 + mc::gamma2) / 36.0;   // M^-1 = M^T diag(.., 1/36, 1/36, ..)
constexpr double v_rest = -4.0 * a1 + 4.0 * a2;
constexpr double v_axis = -a1 - 2.0 * a2;
constexpr double v_diag = 2.0 * a1 + a2;
constexpr double m1 = 4.0 + mc::gamma1, m2 = -4.0 + mc::gamma2;   // rows 1, 2 of M v
constexpr double m3 = 2.0 * v_axis + 4.0 * v_diag;                 // sum_q e_qx^2 v_q
constexpr double m4 = -4.0 * v_axis + 4.0 * v_diag;                // sum_q M_4q e_qx v_q
static_assert(v_rest + 4.0 * v_axis + 4.0 * v_diag == 0.0, "the reference leaves n_0 unchanged");
}  // namespace gref
template <typename Fm> constexpr bool has_gref = Fm::EG == 2;

// Stochastic rounding (lbm_rounding.hpp) of the format's 16-bit rows.
namespace sr {
template <typename Fm> constexpr bool used = Fm::EF == 2 || Fm::EG == 2;
// index of DF row q (0..17) among the 16-bit rows of the format (negative: not 16-bit)
template <typename Fm> constexpr int index(int q) { return Fm::EF == 2 ? q : q - 9; }
// random operand of DF row q stored at (x, y) (wrapped on a periodic axis) in step t
template <typename Fm> __device__ __forceinline__ unsigned operand_of(int x, int y, unsigned t, int q)
{
    if constexpr (!used<Fm>) return 0u;
    if ((q < 9 ? Fm::EF : Fm::EG) != 2) return 0u;
    return operand_at(x, y, t, index<Fm>(q));
}
}  // namespace sr
template <typename C> __device__ __forceinline__ C gref_v(int q)
{
    return C(q == 0 ? gref::v_rest : (q <= 4 ? gref::v_axis : gref::v_diag));
}
// offset of DF q stored in column col
template <typename Fm> __device__ __forceinline__ typename Fm::C gref_offset(const CaseParams& P, int q, int col)
{
    using C = typename Fm::C;
    if constexpr (!has_gref<Fm>) return C(0);
    const Coef<C>& K = coef<C>(P);
    return gref_v<C>(q) * (K.gs0 + K.gsk * C(col));
}

// side indices of a node: x-side (0/1) or -1, y-side (2/3) or -1
__device__ __forceinline__ int side_x(const CaseParams& P, int x)
{
    return P.wall_x ? (x == 0 ? 0 : (x == P.nx - 1 ? 1 : -1)) : -1;
}
__device__ __forceinline__ int side_y(const CaseParams& P, int y)
{
    return P.wall_y ? (y == 0 ? 2 : (y == P.ny - 1 ? 3 : -1)) : -1;
}

// Macros of a node from its pulled moments: off-wall nodes from the DFs,
// wall nodes from the bounce-back completed sums and the prescribed values.
// The x-wall sets the velocity of a corner and its temperature when it is
// Dirichlet; otherwise a Dirichlet y-wall sets the temperature.
template <typename C>
__device__ __forceinline__ double node_state(const CaseParams& P, const Coef<C>& K, int sx, int sy,
                                             const C m[9], C n0, NodeState<C>& s)
{
    if (sx < 0 && sy < 0) return state_from_moments<C>(K, P.eos, P.per_mass, m, n0, s);
    const int sv = sx >= 0 ? sx : sy;
    int adiabatic = 1;
    double Tw = 0.0;
    if (sx >= 0 && !P.side_adiabatic[sx]) { adiabatic = 0; Tw = K.side_T[sx]; }
    else if (sy >= 0 && !P.side_adiabatic[sy]) { adiabatic = 0; Tw = K.side_T[sy]; }
    return state_wall<C>(K, P.eos, P.per_mass, m[0], n0, K.side_ux[sv], K.side_uy[sv],
                         adiabatic, Tw, s);
}

// Pull the 18 DFs of node (x, y) (generic indexing) and take their moments.
template <typename Fm>
__device__ __forceinline__ void pull_node(const CaseParams& P, const char* src, int x, int y,
                                          typename Fm::C m[9], typename Fm::C n[9])
{
    using C = typename Fm::C;
    C f[9], g[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) {
        const int sx = x - EXq(q), sy = y - EYq(q);
        const int slot = col_slot(P, sx);
        f[q] = load_df<Fm>(src, q, row_byte<Fm>(P, q, sy) + slot_bytes<Fm>(q, slot));
        g[q] = load_df<Fm>(src, 9 + q, row_byte<Fm>(P, 9 + q, sy) + slot_bytes<Fm>(9 + q, slot));
        if constexpr (has_gref<Fm>) g[q] += gref_offset<Fm>(P, q, sx);
    }
    to_moments<C>(f, m);
    to_moments<C>(g, n);
}

// store the 18 DFs of node (x, y) into every slot that holds its column
template <typename Fm>
__device__ __forceinline__ void store_node(const CaseParams& P, char* dst, int x, int y,
                                           const typename Fm::C fb[9], const typename Fm::C gb[9], unsigned t)
{
    typename Fm::C gs[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) gs[q] = gb[q] - gref_offset<Fm>(P, q, x);
    for_each_slot(P, x, [&](int slot) {
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            store_df<Fm>(dst, q, row_byte<Fm>(P, q, y) + slot_bytes<Fm>(q, slot), fb[q], sr::operand_of<Fm>(x, y, t, q));
            store_df<Fm>(dst, 9 + q, row_byte<Fm>(P, 9 + q, y) + slot_bytes<Fm>(9 + q, slot), gs[q],
                         sr::operand_of<Fm>(x, y, t, 9 + q));
        }
    });
}

// Write the post-collision DFs of a wall node that leave the domain into the
// ghost cells they reach, in the row of the opposite direction.
template <typename Fm>
__device__ __forceinline__ void store_ghosts(const CaseParams& P, char* dst, int x, int y,
                                             const typename Fm::C fb[9], const typename Fm::C gb[9], unsigned t)
{
#pragma unroll
    for (int q = 1; q < 9; ++q) {
        const int tx = x + EXq(q), ty = y + EYq(q);
        const bool out = (P.wall_x && (tx < 0 || tx >= P.nx)) || (P.wall_y && (ty < 0 || ty >= P.ny));
        if (out) {
            const int qf = OPPq(q), qg = 9 + OPPq(q);
            const typename Fm::C gs = gb[q] - gref_offset<Fm>(P, OPPq(q), tx);
            const int kx = wrap_axis(tx, P.nx, P.wall_x), ky = wrap_axis(ty, P.ny, P.wall_y);
            const unsigned uf = sr::operand_of<Fm>(kx, ky, t, qf), ug = sr::operand_of<Fm>(kx, ky, t, qg);
            for_each_slot(P, tx, [&](int slot) {
                store_df<Fm>(dst, qf, row_byte<Fm>(P, qf, ty) + slot_bytes<Fm>(qf, slot), fb[q], uf);
                store_df<Fm>(dst, qg, row_byte<Fm>(P, qg, ty) + slot_bytes<Fm>(qg, slot), gs, ug);
            });
        }
    }
}

template <typename C>
__device__ __forceinline__ void export_node(const CaseParams& P, int x, int y, const NodeState<C>& s, double T_d)
{
    const Coef<C>& K = coef<C>(P);
    const long long nn = (long long)P.nx * P.ny;
    const long long i = (long long)y * P.nx + x;
    const double rho = K.rho0_d + double(s.drho);
    P.macro[i] = rho;
    P.macro[nn + i] = double(s.ux);
    P.macro[2 * nn + i] = double(s.uy);
    P.macro[3 * nn + i] = T_d;
    P.macro[4 * nn + i] = K.p0_d + double(s.dp);
    const bool ok = rho > 0.0 && T_d > 0.0 && rho < 1e30 && T_d < 1e30 && s.ux == s.ux && s.uy == s.uy &&
                    s.dp == s.dp;
    if (!ok) atomicOr(P.flag, 1);
}

// ---------------------------------------------------------------------------
// collision of an off-wall node given its pulled moments, written so that
// the temporaries of the f part are dead before the g part starts:
//   N = m - m^eq + F_m/2, Ntil = (I - S/2) N,
//   mbar = 2 m^eq - m + 2 Ntil - [R Ntil + T.grad rho + X.grad p]
//   (eq. LBE.u.c with m = m^eq - F_m/2 + N), conserved rows mbar_0 = m_0,
//   mbar_3 = m_3 + F_x, mbar_5 = m_5 + F_y;
//   H = n - n^eq + Q_m/2, Htil = (I - L/2) H (App. C steps 1-3),
//   nbar = 2 n^eq - n + 2 Htil + Y [(m + mbar)/2 - m^eq] (eq. LBE.T.c,
//   App. C step 4), conserved row nbar_0 = n_0 + q_e.
// The f and g post-collision deviations go to fb and gb; gb is taken
// relative to the 16-bit reference of the node's column (sref, zero without
// one).
// ---------------------------------------------------------------------------
// Whole-wavefront lane shifts by one lane (DPP wave_shr:1 / wave_shl:1):
// lane l receives the value of lane l - 1 (from_left) or l + 1 (from_right);
// lane 0, resp. 63, receives 0.  Every lane of the wavefront must be active.
constexpr int kDppWaveShl1 = 0x130, kDppWaveShr1 = 0x138;
template <int CTRL>
__device__ __forceinline__ int dpp_shift(int v)
{
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp_shift(float v)
{
    return __int_as_float(dpp_shift<CTRL>(__float_as_int(v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp_shift(double v)
{
    const unsigned long long u = __builtin_bit_cast(unsigned long long, v);
    const unsigned lo = unsigned(dpp_shift<CTRL>(int(unsigned(u)))), hi = unsigned(dpp_shift<CTRL>(int(unsigned(u >> 32))));
    return __builtin_bit_cast(double, (unsigned long long)lo | ((unsigned long long)hi << 32));
}
template <typename C>
__device__ __forceinline__ C from_left(C v) { return dpp_shift<kDppWaveShr1>(v); }
template <typename C>
__device__ __forceinline__ C from_right(C v) { return dpp_shift<kDppWaveShl1>(v); }

// Lanes of a strip that holds an x-wall column collide the wall node there
// (Sec. 3.1): its non-equilibrium part is not its own but the tilde moments
// of the off-wall nodes x_f = x_w + n and x_ff = x_w + 2n along the inner
// normal n, extrapolated to first or second order (eq. neq.extrapolation,
// Zm = Ntil(x_f) [2 Ntil(x_f) - Ntil(x_ff)], Zn likewise from
// Htil + (Y/2) Ntil), and inverted with the wall node's own S, L and Y
// (App. B).  x_f and x_ff are collided by the neighbouring lanes of the same
// row, whose tilde moments are read by lane permutation.
struct XWallLane {
    bool wall;       // this lane collides a wall node
    bool left;       // ... of the left wall (x_f, x_ff on the lanes above it; else below)
    bool order2;     // second-order extrapolation
};

template <typename C>
__device__ __forceinline__ C lane_extrap(C v, const XWallLane& xl)
{
    // both directions are shifted by every lane before a lane selects one
    const C r1 = from_right(v), l1 = from_left(v);
    const C a = xl.left ? r1 : l1;
    if (!xl.order2) return a;
    const C r2 = from_right(r1), l2 = from_left(l1);
    return C(2) * a - (xl.left ? r2 : l2);
}

// With XW, the wall lanes of the row take the extrapolated pair: with
// Ntil := Zm, N := (I - S/2)^-1 Zm, Htil := Zn - (Y/2) Zm, H := (I - L/2)^-1 Htil
// and m := m^eq - F_m/2 + N, n := n^eq - Q_m/2 + H substituted, the update
// below is the post-collision state of the wall node.  The lanes of x_f and
// x_ff are off-wall lanes, so their Ntil and Htil are their own when the
// wall lanes read them.
template <typename C, bool XW = false>
__device__ __forceinline__ void collide_interior(const CaseParams& P, const Coef<C>& K, const NodeState<C>& s,
                                                 const C m[9], const C n[9],
                                                 C gr_x, C gr_y, C gp_x, C gp_y, C fb[9], C gb[9],
                                                 C sref,
                                                 const XWallLane& xl = XWallLane{false, false, false})
{
    Rates<C> r;
    local_rates<C>(K, P.visc_law, s, r);
    const Forcing<C> F = forcing<C>(K, P.per_mass, s);
    C G1, G7, G8;
    C y3 = C(0), y5 = C(0);   // (Y/2)-part of Htil from this lane's u and Ntil (XW)
    {
        C meq[9], N[9], Nt[9], mb[9], mm[9];
        {
            C Fm[9];
            meq_f<C>(s, meq);
            force_moments<C>(s, F, Fm);
#pragma unroll
            for (int i = 0; i < 9; ++i) N[i] = m[i] - meq[i] + C(0.5) * Fm[i];
            N[0] = C(0);
            N[3] = C(0);
            N[5] = C(0);
            tilde_f<C>(s, r, N, Nt);
#pragma unroll
            for (int i = 0; i < 9; ++i) mm[i] = m[i];
            if constexpr (XW) {
                // every lane takes part in the permutations (a lane reading
                // from a lane switched off by a branch would read nothing)
#pragma unroll
                for (int i = 0; i < 9; ++i) {
                    if (i == 0 || i == 3 || i == 5) continue;
                    const C z = lane_extrap<C>(Nt[i], xl);
                    Nt[i] = xl.wall ? z : Nt[i];
                }
                untilde_f<C>(s, r, Nt, N);
                C Fw[9];
                force_moments<C>(s, F, Fw);
#pragma unroll
                for (int i = 0; i < 9; ++i) mm[i] = xl.wall ? meq[i] - C(0.5) * Fw[i] + N[i] : m[i];
                y3 = s.ux * (C(1.0 / 3.0) * Nt[1] + Nt[7]) + C(2) * s.uy * Nt[8];
                y5 = s.uy * (C(1.0 / 3.0) * Nt[1] - Nt[7]) + C(2) * s.ux * Nt[8];
            }
        }
        C c1, c7, c8;
        corrections<C>(s, r, P.cubic, Nt, gr_x, gr_y, gp_x, gp_y, c1, c7, c8);
#pragma unroll
        for (int i = 0; i < 9; ++i) mb[i] = C(2) * meq[i] - mm[i] + C(2) * Nt[i];
        mb[0] = mm[0];
        mb[3] = mm[3] + F.Fx;
        mb[5] = mm[5] + F.Fy;
        mb[1] -= c1;
        mb[7] -= c7;
        mb[8] -= c8;
        // (m + mbar)/2 - m^eq on rows 1, 7, 8
        G1 = Nt[1] - C(0.5) * c1;
        G7 = Nt[7] - C(0.5) * c7;
        G8 = Nt[8] - C(0.5) * c8;
        from_moments<C>(mb, fb);
    }
    {
        C neq[9], Hm[9], Ht[9], nb[9], nn[9];
        {
            C Qm[9];
            neq_g<C>(K, s, neq);
            source_moments<C>(s, F, Qm);
#pragma unroll
            for (int i = 0; i < 9; ++i) Hm[i] = n[i] - neq[i] + C(0.5) * Qm[i];
            Hm[0] = C(0);
            tilde_g<C>(r, Hm, Ht);
#pragma unroll
            for (int i = 0; i < 9; ++i) nn[i] = n[i];
            if constexpr (XW) {
                // Zn = Htil + (Y/2) Ntil of the off-wall lanes, extrapolated;
                // the wall's Htil = Zn - (Y/2) Zm with the wall velocity
#pragma unroll
                for (int i = 1; i < 9; ++i) {
                    const C ys = i == 3 || i == 4 ? y3 : (i == 5 || i == 6 ? y5 : C(0));
                    const C sgn = i == 3 || i == 5 ? C(0.5) : C(-0.5);
                    const C zo = (i >= 3 && i <= 6) ? Ht[i] + sgn * ys : Ht[i];
                    const C zw = lane_extrap<C>(zo, xl);
                    Ht[i] = xl.wall ? ((i >= 3 && i <= 6) ? zw - sgn * ys : zw) : Ht[i];
                }
                untilde_g<C>(r, Ht, Hm);
                C Qw[9];
                source_moments<C>(s, F, Qw);
#pragma unroll
                for (int i = 0; i < 9; ++i) nn[i] = xl.wall ? neq[i] - C(0.5) * Qw[i] + Hm[i] : n[i];
            }
        }
#pragma unroll
        for (int i = 0; i < 9; ++i) nb[i] = C(2) * neq[i] - nn[i] + C(2) * Ht[i];
        nb[0] = nn[0] + F.qe;
        const C z3 = s.ux * (C(1.0 / 3.0) * G1 + G7) + C(2) * s.uy * G8;
        const C z5 = s.uy * (C(1.0 / 3.0) * G1 - G7) + C(2) * s.ux * G8;
        nb[3] += z3;
        nb[4] -= z3;
        nb[5] += z5;
        nb[6] -= z5;
        // stored g: measured from the 16-bit rows' reference of this column
        nb[1] -= C(gref::m1) * sref;
        nb[2] -= C(gref::m2) * sref;
        from_moments<C>(nb, gb);
    }
}

// ---------------------------------------------------------------------------
// interior item: march up a strip segment
// ---------------------------------------------------------------------------
// Wave priority from progress: a wavefront that has done less of its rows
// is issued first, so the waves of a CU advance together and finish close to
// each other instead of leaving a few young waves to run alone at the end.
template <typename Fm>
__device__ __forceinline__ void progress_priority(int done, int total)
{
    if constexpr (Tuning<Fm>::fair) {
        const int q = (4 * done) / total;      // 0..3 for done < total
        if (q == 0) __builtin_amdgcn_s_setprio(3);
        else if (q == 1) __builtin_amdgcn_s_setprio(2);
        else if (q == 2) __builtin_amdgcn_s_setprio(1);
        else __builtin_amdgcn_s_setprio(0);
    }
}

// stored row (0 .. ny+1) of lattice row v in [-1, ny], wrapped on a periodic axis
__device__ __forceinline__ int stored_row(int v, int n, int walled)
{
    if (!walled) {
        v %= n;
        if (v < 0) v += n;
    }
    return v + 1;
}

// interior item: the 64 lanes take the 64 slots of one strip region, i.e.
// columns X - 1 .. X + 62 of a strip whose own columns are X .. X + 61, and
// march up the rows [y0, y0 + len).  Lanes 1..62 collide the strip's own
// nodes (their x-neighbours are lanes 0..63); lanes 0 and 63 only provide
// the state of the neighbouring strips' edge columns for the gradients, and
// on a walled x axis a lane on a wall column collides the wall node when the
// strip takes it (XW).  All memory traffic goes
// through buffer resources: one per stored row block, per-lane byte offsets
// of the source slots in VGPRs, the DF row inside the block as a scalar
// offset.  The loop body has no divergent branch: lanes whose slot must not
// be written get an offset past the record count, which the hardware drops,
// so the loads of row y + 2 stay in flight across the collision and the
// stores of row y.
template <typename Fm, bool EXPORT, bool XW>
__device__ __forceinline__ void interior_item(const CaseParams& P, const WorkItem w, const char* __restrict__ src_in,
                                              char* __restrict__ dst_in, typename Fm::C* __restrict__ park,
                                              unsigned tk)
{
    const char* __restrict__ src = uniform_ptr(src_in);
    char* __restrict__ dst = uniform_ptr(dst_in);
    using C = typename Fm::C;
    using F = typename Fm::F;
    using G = typename Fm::G;
    constexpr int EF = Fm::EF, EG = Fm::EG;
    const Coef<C>& K = coef<C>(P);
    const int lane = threadIdx.x & (WAVE - 1);
    const int nx = P.nx, ny = P.ny, pitch = P.pitch;
    const int wall_x = P.wall_x, wall_y = P.wall_y;
    const int xhi = wall_x ? nx - 1 : nx;          // end of the off-wall columns
    const int X = w.x0;                            // first own column
    const int region = (X - P.xlo) / STRIP_COLS * REGION_SLOTS;
    const int c = X - 1 + lane;                    // column of this lane's slot
    // the node this lane collides: its column, held inside [0, nx) on a walled axis
    const int cn = wall_x ? min(max(c, 0), nx - 1) : wrap_axis(c, nx, 0);
    const bool regular = c == cn || !wall_x;
    const int sx = side_x(P, cn);
    const unsigned sx_seed = sr::seed_x(cn);   // column part of the stochastic-rounding seed
    // reference of 16-bit g rows: s at this lane's node column (its moments
    // in rows 1 and 2 are m1 s and m2 s) and the part that a pull from the
    // neighbouring columns adds to rows 3 and 4 (wave-uniform); zero without
    // a reference
    C sref = C(0), gr3 = C(0), gr4 = C(0);
    if constexpr (has_gref<Fm>) {
        sref = K.gs0 + K.gsk * C(cn);
        gr3 = C(-gref::m3) * K.gsk;
        gr4 = C(-gref::m4) * K.gsk;
    }
    // slot a pull along e_x reads: inside the own region for this strip's own
    // columns, the owning slot (col_slot) for the neighbouring strips'
    // columns and the wall, ghost and wrapped columns
    auto src_slot = [&](int ex) {
        const int d = c - ex, p = d - (X - 1);
        const bool inside = regular && p >= 1 && p <= STRIP_COLS && d >= P.xlo && d < xhi;
        return inside ? region + p : col_slot(P, cn - ex);
    };
    const int sl0 = src_slot(1), sl1 = src_slot(0), sl2 = src_slot(-1);
    // per-lane byte offsets in f rows and in g rows (the same when both use one type)
    const int vf0 = sl0 * EF, vf1 = sl1 * EF, vf2 = sl2 * EF;
    const int vg0 = sl0 * EG, vg1 = sl1 * EG, vg2 = sl2 * EG;
    // x-wall nodes collided by this strip (XW: the case has them in its
    // strips and this strip holds the column 0 or nx - 1 on a lane 1..62)
    XWallLane xl{false, false, P.extrap_order == 2};
    if constexpr (XW) {
        xl.left = c == 0;
        xl.wall = c == 0 || c == nx - 1;
    }
    // the strip holds the left / right wall column (wave-uniform)
    const bool has_left = XW && X == P.xlo, has_right = XW && X + STRIP_COLS >= nx - 1;   // lanes 0 .. 63 reach X + 62
    // slots this lane stores: the whole region, so that every store covers
    // whole cache lines (a partly written line costs the memory system a
    // read-modify-write), except the wall and ghost slots of a walled side,
    // unless the lane collides the wall node, and the slots past the end of
    // a ragged last strip.  The halo lanes 0 and 63 write slots that nothing
    // reads.
    const bool keep = !xl.wall && (wall_x ? (c < P.xlo || c >= xhi) : c > nx);
    const int vf_out = keep ? kDropOffset : (region + lane) * EF;
    const int vg_out = keep ? kDropOffset : (region + lane) * EG;
    const bool out_lane = lane >= 1 && lane <= STRIP_COLS && c >= P.xlo && c < xhi;   // own nodes
    const int frow_bytes = pitch * EF, grow_bytes = pitch * EG, g_base = 9 * frow_bytes;
    const unsigned blk_bytes = unsigned(9 * (frow_bytes + grow_bytes));
    const long long blk = blk_bytes;
    const int ylast_row = w.y0 + w.len - 1;

    // pull lattice row yy: DF q comes from (x - e_qx, yy - e_qy)
    auto pull = [&](int yy, C f[9], C g[9]) {
        const rsrc_t r_s = make_rsrc(src + stored_row(yy - 1, ny, wall_y) * blk, blk_bytes);
        const rsrc_t r_c = make_rsrc(src + stored_row(yy, ny, wall_y) * blk, blk_bytes);
        const rsrc_t r_n = make_rsrc(src + stored_row(yy + 1, ny, wall_y) * blk, blk_bytes);
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            const rsrc_t r = EYq(q) == 1 ? r_s : (EYq(q) == 0 ? r_c : r_n);
            const int vf = EXq(q) == 1 ? vf0 : (EXq(q) == 0 ? vf1 : vf2);
            const int vg = EXq(q) == 1 ? vg0 : (EXq(q) == 0 ? vg1 : vg2);
            f[q] = Store<F>::bload(r, vf, q * frow_bytes);
            g[q] = Store<G>::bload(r, vg, g_base + q * grow_bytes);
        }
    };
    // A strip next to an x-wall has lanes on the wall column; their state
    // takes the wall velocity / temperature by selection (no divergence).
    const bool edge = Tuning<Fm>::edge_select && wall_x && (X - 1 <= 0 || X + STRIP_COLS >= nx - 1);
    // moments and state of a pulled row (wall rows: uniform branch to the wall formulas)
    auto row_state = [&](int yy, const C f[9], const C g[9], C dm[9], C dn[9], NodeState<C>& st) {
        to_moments<C>(f, dm);
        to_moments<C>(g, dn);
        if constexpr (has_gref<Fm>) {
            dn[1] += C(gref::m1) * sref;
            dn[2] += C(gref::m2) * sref;
            dn[3] += gr3;
            if constexpr (gref::m4 != 0.0) dn[4] += gr4;
        }
        const int sy = side_y(P, stored_row(yy, ny, wall_y) - 1);
        if (sy >= 0 || !Tuning<Fm>::edge_select) return node_state<C>(P, K, sx, sy, dm, dn[0], st);
        if (edge) {
            const bool right = sx == 1;
            const bool dir = sx >= 0 && !(right ? P.side_adiabatic[1] : P.side_adiabatic[0]);
            return state_select<C>(K, P.eos, P.per_mass, dm, dn[0], sx >= 0, right ? K.side_ux[1] : K.side_ux[0],
                                   right ? K.side_uy[1] : K.side_uy[0], dir, right ? K.side_T[1] : K.side_T[0], st);
        }
        return state_from_moments<C>(K, P.eos, P.per_mass, dm, dn[0], st);
    };

    // March direction: segments alternate up (d = +1) and down (d = -1), so
    // the two rows a segment boundary shares are pulled by both segments at
    // the same moment (both at the start or both at the end of the step).
    // "ahead" is the next row in the direction of the march, "behind" the
    // previous one.
    const int d = Tuning<Fm>::alternate && w.dir ? -1 : 1;
    const int yf = d > 0 ? w.y0 : ylast_row;
    C m_c[9], n_c[9], m_n[9], n_n[9];
    NodeState<C> s_c, s_n;          // current row, row ahead
    C rho_b, p_b;                   // row behind
    {
        C f[9], g[9], dm[9], dn[9];
        NodeState<C> st;
        pull(yf - d, f, g);
        row_state(yf - d, f, g, dm, dn, st);
        rho_b = st.drho;
        p_b = st.dp;
        pull(yf, f, g);
        row_state(yf, f, g, m_c, n_c, s_c);
        pull(yf + d, f, g);
        row_state(yf + d, f, g, m_n, n_n, s_n);
    }
    // The moments of the row ahead are not used before the next row: they
    // wait in this wavefront's LDS slice, so that the collision of the
    // current row has their registers.
    auto park_store = [&](const C m[9], const C n[9]) {
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            park[q * WAVE + lane] = m[q];
            park[(9 + q) * WAVE + lane] = n[q];
        }
    };
    if constexpr (Tuning<Fm>::park) park_store(m_n, n_n);

    for (int i = 0; i < w.len; ++i) {
        if constexpr (Tuning<Fm>::lockstep) __syncthreads();
        progress_priority<Fm>(i, w.len);
        const int y = yf + i * d;
        // loads of the row two ahead (on the last row a repeat of the row
        // ahead, which is in cache and whose state is not used) before the
        // collision
        const int ynext = i + 1 < w.len ? y + 2 * d : y + d;
        C fr[9], gr[9];
        if constexpr (!XW || Tuning<Fm>::xw_prefetch) pull(ynext, fr, gr);

        // isotropic gradients d_a phi = 3 sum_q w_q e_qa phi(x + e_q), taken on
        // the deviations rho - rho0 and p - p0, written symmetric in ahead /
        // behind so that both march directions round alike
        const C rW = from_left(s_c.drho), rE = from_right(s_c.drho);
        const C rBW = from_left(rho_b), rBE = from_right(rho_b);
        const C rAW = from_left(s_n.drho), rAE = from_right(s_n.drho);
        const C pW = from_left(s_c.dp), pE = from_right(s_c.dp);
        const C pBW = from_left(p_b), pBE = from_right(p_b);
        const C pAW = from_left(s_n.dp), pAE = from_right(s_n.dp);
        const C fd = C(d);
        const C gr_x = (rE - rW) * C(1.0 / 3.0) + ((rAE - rAW) + (rBE - rBW)) * C(1.0 / 12.0);
        const C gr_y = fd * ((s_n.drho - rho_b) * C(1.0 / 3.0) + ((rAE + rAW) - (rBE + rBW)) * C(1.0 / 12.0));
        const C gp_x = (pE - pW) * C(1.0 / 3.0) + ((pAE - pAW) + (pBE - pBW)) * C(1.0 / 12.0);
        const C gp_y = fd * ((s_n.dp - p_b) * C(1.0 / 3.0) + ((pAE + pAW) - (pBE + pBW)) * C(1.0 / 12.0));

        C fb[9], gb[9];
        if constexpr (XW) {
            // gradients at a wall node: second-order one-sided along x from
            // x_f and x_ff, two-point central along y
            const C r1 = xl.left ? rE : rW, p1 = xl.left ? pE : pW;
            const C rEE = from_right(rE), rWW = from_left(rW), pEE = from_right(pE), pWW = from_left(pW);
            const C r2 = xl.left ? rEE : rWW, p2 = xl.left ? pEE : pWW;
            const C sg = xl.left ? C(1) : C(-1);
            const C wr_x = sg * ((C(-3) * s_c.drho + C(4) * r1 - r2) * C(0.5));
            const C wp_x = sg * ((C(-3) * s_c.dp + C(4) * p1 - p2) * C(0.5));
            const C wr_y = fd * ((s_n.drho - rho_b) * C(0.5));
            const C wp_y = fd * ((s_n.dp - p_b) * C(0.5));
            collide_interior<C, true>(P, K, s_c, m_c, n_c, xl.wall ? wr_x : gr_x, xl.wall ? wr_y : gr_y,
                                      xl.wall ? wp_x : gp_x, xl.wall ? wp_y : gp_y, fb, gb, sref, xl);
        } else {
            collide_interior<C>(P, K, s_c, m_c, n_c, gr_x, gr_y, gp_x, gp_y, fb, gb, sref);
        }
        const rsrc_t ro = make_rsrc(dst + (long long)(y + 1) * blk, blk_bytes);
        if constexpr (sr::used<Fm>) {
            // the f rows, then the g rows, so that few random words are live at once
            unsigned w = sr::mix(sx_seed ^ sr::seed_yt(y, tk));   // word 0 of this lane's node
            int wk = 0;
#pragma unroll
            for (int j = 0; j < 18; ++j) {
                const int q = j < 9 ? j : j - 9;
                const int i = sr::index<Fm>(j);
                if (i < 0) {
                    Store<F>::bstore(ro, vf_out, q * frow_bytes, fb[q]);
                    continue;
                }
                if (i / sr::kOperandsPerWord != wk) {
                    w = sr::xorshift(w);
                    wk = i / sr::kOperandsPerWord;
                }
                const unsigned rnd = sr::rotl(w, sr::kOperandShift * (i % sr::kOperandsPerWord));
                if (j < 9) Store<F>::bstore_sr(ro, vf_out, q * frow_bytes, fb[q], rnd);
                else Store<G>::bstore_sr(ro, vg_out, g_base + q * grow_bytes, gb[q], rnd);
            }
        } else {
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                Store<F>::bstore(ro, vf_out, q * frow_bytes, fb[q]);
                Store<G>::bstore(ro, vg_out, g_base + q * grow_bytes, gb[q]);
            }
        }
        if constexpr (XW) {
            // the DFs a wall node sends out of the domain go to the ghost
            // column next to it, in the row they reach and as the opposite
            // direction (the bounce-back of the next pull)
            const rsrc_t rp = make_rsrc(dst + (long long)stored_row(y + 1, ny, wall_y) * blk, blk_bytes);
            const rsrc_t rm = make_rsrc(dst + (long long)stored_row(y - 1, ny, wall_y) * blk, blk_bytes);
            const int gsl = col_slot(P, xl.left ? -1 : c + 1);   // the wall lane's ghost slot
            // gb is relative to the 16-bit reference of the wall column; the
            // ghost column next to it (x -/+ 1) has offsets v_q gsk higher / lower
            C gka = C(0), gkd = C(0);
            if constexpr (has_gref<Fm>) {
                gka = C(gref::v_axis) * K.gsk;
                gkd = C(gref::v_diag) * K.gsk;
            }
            // random operands of the ghost slots (column x -/+ 1, rows y, y + 1, y - 1)
            const int gcol = xl.left ? c - 1 : c + 1;
            const int yp = wrap_axis(y + 1, ny, wall_y), ym = wrap_axis(y - 1, ny, wall_y);
            if (has_left) {
                // left wall: q = 3, 6, 7 leave as 1, 8, 5 in rows y, y + 1, y - 1
                const int vf = xl.wall && xl.left ? gsl * EF : kDropOffset, vg = xl.wall && xl.left ? gsl * EG : kDropOffset;
                Store<F>::bstore_sr(ro, vf, 1 * frow_bytes, fb[3], sr::operand_of<Fm>(gcol, y, tk, 1));
                Store<G>::bstore_sr(ro, vg, g_base + 1 * grow_bytes, gb[3] + gka, sr::operand_of<Fm>(gcol, y, tk, 10));
                Store<F>::bstore_sr(rp, vf, 8 * frow_bytes, fb[6], sr::operand_of<Fm>(gcol, yp, tk, 8));
                Store<G>::bstore_sr(rp, vg, g_base + 8 * grow_bytes, gb[6] + gkd, sr::operand_of<Fm>(gcol, yp, tk, 17));
                Store<F>::bstore_sr(rm, vf, 5 * frow_bytes, fb[7], sr::operand_of<Fm>(gcol, ym, tk, 5));
                Store<G>::bstore_sr(rm, vg, g_base + 5 * grow_bytes, gb[7] + gkd, sr::operand_of<Fm>(gcol, ym, tk, 14));
            }
            if (has_right) {
                // right wall: q = 1, 5, 8 leave as 3, 7, 6 in rows y, y + 1, y - 1
                const int vf = xl.wall && !xl.left ? gsl * EF : kDropOffset, vg = xl.wall && !xl.left ? gsl * EG : kDropOffset;
                Store<F>::bstore_sr(ro, vf, 3 * frow_bytes, fb[1], sr::operand_of<Fm>(gcol, y, tk, 3));
                Store<G>::bstore_sr(ro, vg, g_base + 3 * grow_bytes, gb[1] - gka, sr::operand_of<Fm>(gcol, y, tk, 12));
                Store<F>::bstore_sr(rp, vf, 7 * frow_bytes, fb[5], sr::operand_of<Fm>(gcol, yp, tk, 7));
                Store<G>::bstore_sr(rp, vg, g_base + 7 * grow_bytes, gb[5] - gkd, sr::operand_of<Fm>(gcol, yp, tk, 16));
                Store<F>::bstore_sr(rm, vf, 6 * frow_bytes, fb[8], sr::operand_of<Fm>(gcol, ym, tk, 6));
                Store<G>::bstore_sr(rm, vg, g_base + 6 * grow_bytes, gb[8] - gkd, sr::operand_of<Fm>(gcol, ym, tk, 15));
            }
        }
        if (EXPORT && (out_lane || xl.wall)) export_node<C>(P, c, y, s_c, K.T0_d + double(s_c.dT));
        rho_b = s_c.drho;
        p_b = s_c.dp;
        s_c = s_n;
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            m_c[q] = Tuning<Fm>::park ? park[q * WAVE + lane] : m_n[q];
            n_c[q] = Tuning<Fm>::park ? park[(9 + q) * WAVE + lane] : n_n[q];
        }
        if constexpr (XW && !Tuning<Fm>::xw_prefetch) pull(ynext, fr, gr);
        row_state(ynext, fr, gr, m_n, n_n, s_n);
        if constexpr (Tuning<Fm>::park) park_store(m_n, n_n);
    }
}

// ---------------------------------------------------------------------------
// wall item
// ---------------------------------------------------------------------------
// Wall nodes a case gives to wall items, enumerated as: bottom row, top row
// (walled y, corners included), then, when the strips next to the x-walls
// do not collide them, the left and right columns between those rows.
__device__ __forceinline__ void wall_node_xy(const CaseParams& P, int i, int& x, int& y)
{
    if (P.wall_y) {
        if (i < P.nx) { x = i; y = 0; return; }
        i -= P.nx;
        if (i < P.nx) { x = i; y = P.ny - 1; return; }
        i -= P.nx;
    }
    const int ylo = P.wall_y ? 1 : 0, len = P.wall_y ? P.ny - 2 : P.ny;
    x = i < len ? 0 : P.nx - 1;
    y = ylo + (i < len ? i : i - len);
}

template <typename Fm>
__device__ __forceinline__ typename Fm::C node_rho_p(const CaseParams& P, const char* src, int x, int y,
                                                    typename Fm::C& p)
{
    using C = typename Fm::C;
    C m[9], n[9];
    NodeState<C> s;
    pull_node<Fm>(P, src, x, y, m, n);
    const int xw = wrap_axis(x, P.nx, P.wall_x), yw = wrap_axis(y, P.ny, P.wall_y);
    node_state<C>(P, coef<C>(P), side_x(P, xw), side_y(P, yw), m, n[0], s);
    p = s.dp;
    return s.drho;
}

// derivative of rho and p (as deviations) along one axis at a wall node (second-order
// one-sided towards the inside along a walled axis it lies on, two-point
// central otherwise)
template <typename Fm>
__device__ __forceinline__ void wall_axis_gradient(const CaseParams& P, const char* src, int x, int y, int ax,
                                                   typename Fm::C rho0, typename Fm::C p0,
                                                   typename Fm::C& gr, typename Fm::C& gp)
{
    using C = typename Fm::C;
    const int dx = ax == 0 ? 1 : 0, dy = ax == 0 ? 0 : 1;
    const int s = ax == 0 ? side_x(P, x) : side_y(P, y);
    C p1, p2;
    if (s == 0 || s == 2) {
        const C r1 = node_rho_p<Fm>(P, src, x + dx, y + dy, p1);
        const C r2 = node_rho_p<Fm>(P, src, x + 2 * dx, y + 2 * dy, p2);
        gr = (C(-3) * rho0 + C(4) * r1 - r2) * C(0.5);
        gp = (C(-3) * p0 + C(4) * p1 - p2) * C(0.5);
    } else if (s == 1 || s == 3) {
        const C r1 = node_rho_p<Fm>(P, src, x - dx, y - dy, p1);
        const C r2 = node_rho_p<Fm>(P, src, x - 2 * dx, y - 2 * dy, p2);
        gr = (C(3) * rho0 - C(4) * r1 + r2) * C(0.5);
        gp = (C(3) * p0 - C(4) * p1 + p2) * C(0.5);
    } else {
        const C r1 = node_rho_p<Fm>(P, src, x + dx, y + dy, p1);
        const C r2 = node_rho_p<Fm>(P, src, x - dx, y - dy, p2);
        gr = (r1 - r2) * C(0.5);
        gp = (p1 - p2) * C(0.5);
    }
}

// Tilde non-equilibrium moments of an off-wall node (eq. neq.redefinition):
//   Zm = (I - S/2) m^neq,  Zn = (I - L/2) n^neq + (Y/2) Zm
template <typename Fmt>
__device__ __forceinline__ void tilde_at(const CaseParams& P, const char* src, int x, int y,
                                         typename Fmt::C Zm[9], typename Fmt::C Zn[9])
{
    using C = typename Fmt::C;
    const Coef<C>& K = coef<C>(P);
    C m[9], n[9];
    NodeState<C> s;
    pull_node<Fmt>(P, src, x, y, m, n);
    node_state<C>(P, K, -1, -1, m, n[0], s);
    Rates<C> r;
    local_rates<C>(K, P.visc_law, s, r);
    const Forcing<C> F = forcing<C>(K, P.per_mass, s);
    C meq[9], Fm[9], neq[9], Qm[9], N[9], Hm[9];
    meq_f<C>(s, meq);
    force_moments<C>(s, F, Fm);
    neq_g<C>(K, s, neq);
    source_moments<C>(s, F, Qm);
    nonequilibrium<C>(s, r, m, n, meq, Fm, neq, Qm, N, Zm, Hm, Zn);
    const C y3 = s.ux * (C(1.0 / 3.0) * Zm[1] + Zm[7]) + C(2) * s.uy * Zm[8];
    const C y5 = s.uy * (C(1.0 / 3.0) * Zm[1] - Zm[7]) + C(2) * s.ux * Zm[8];
    Zn[3] += C(0.5) * y3;
    Zn[4] -= C(0.5) * y3;
    Zn[5] += C(0.5) * y5;
    Zn[6] -= C(0.5) * y5;
}

// One wall node (index i of the case's wall-node enumeration) per lane.
template <typename Fmt, bool EXPORT>
__device__ __forceinline__ void wall_node(const CaseParams& P, int i, const char* __restrict__ src,
                                          char* __restrict__ dst, unsigned tk)
{
    using C = typename Fmt::C;
    const Coef<C>& K = coef<C>(P);
    int xb, yb;
    wall_node_xy(P, i, xb, yb);
    const int sx = side_x(P, xb), sy = side_y(P, yb);

    // macros of the wall node from the bounce-back completed DFs (Sec. 3.1)
    C m[9], n[9];
    NodeState<C> s;
    pull_node<Fmt>(P, src, xb, yb, m, n);
    const double T_d = node_state<C>(P, K, sx, sy, m, n[0], s);

    // extrapolated tilde non-equilibrium moments (eq. neq.extrapolation)
    const int ndx = sx == 0 ? 1 : (sx == 1 ? -1 : 0);
    const int ndy = sy == 2 ? 1 : (sy == 3 ? -1 : 0);
    C Zm[9], Zn[9];
    tilde_at<Fmt>(P, src, xb + ndx, yb + ndy, Zm, Zn);
    if (P.extrap_order == 2) {
        C Zm2[9], Zn2[9];
        tilde_at<Fmt>(P, src, xb + 2 * ndx, yb + 2 * ndy, Zm2, Zn2);
#pragma unroll
        for (int q = 0; q < 9; ++q) {
            Zm[q] = C(2) * Zm[q] - Zm2[q];
            Zn[q] = C(2) * Zn[q] - Zn2[q];
        }
    }
    Zm[0] = C(0);
    Zm[3] = C(0);
    Zm[5] = C(0);
    Zn[0] = C(0);

    // invert with the wall node's own S, L, Y (App. B)
    Rates<C> r;
    local_rates<C>(K, P.visc_law, s, r);
    C N[9], Ht[9], Hm[9];
    untilde_f<C>(s, r, Zm, N);
    {
        const C y3 = s.ux * (C(1.0 / 3.0) * Zm[1] + Zm[7]) + C(2) * s.uy * Zm[8];
        const C y5 = s.uy * (C(1.0 / 3.0) * Zm[1] - Zm[7]) + C(2) * s.ux * Zm[8];
#pragma unroll
        for (int q = 0; q < 9; ++q) Ht[q] = Zn[q];
        Ht[3] -= C(0.5) * y3;
        Ht[4] += C(0.5) * y3;
        Ht[5] -= C(0.5) * y5;
        Ht[6] += C(0.5) * y5;
    }
    untilde_g<C>(r, Ht, Hm);

    // gradients at the wall node
    C gr_x, gr_y, gp_x, gp_y;
    wall_axis_gradient<Fmt>(P, src, xb, yb, 0, s.drho, s.dp, gr_x, gp_x);
    wall_axis_gradient<Fmt>(P, src, xb, yb, 1, s.drho, s.dp, gr_y, gp_y);

    const Forcing<C> F = forcing<C>(K, P.per_mass, s);
    C meq[9], Fm[9], neq[9], Qm[9], mb[9], nb[9], fb[9], gb[9];
    meq_f<C>(s, meq);
    force_moments<C>(s, F, Fm);
    neq_g<C>(K, s, neq);
    source_moments<C>(s, F, Qm);
    post_collision<C>(s, r, P.cubic, meq, Fm, N, Zm, neq, Qm, Hm, Ht, gr_x, gr_y, gp_x, gp_y, mb, nb);
    from_moments<C>(mb, fb);
    from_moments<C>(nb, gb);
    store_node<Fmt>(P, dst, xb, yb, fb, gb, tk);
    store_ghosts<Fmt>(P, dst, xb, yb, fb, gb, tk);
    if (EXPORT) export_node<C>(P, xb, yb, s, T_d);
}

// wall item: wall nodes [x0, x0 + len), 64 at a time
template <typename Fmt, bool EXPORT>
__device__ __forceinline__ void wall_item(const CaseParams& P, const WorkItem w, const char* __restrict__ src,
                                          char* __restrict__ dst, unsigned tk)
{
    const int lane = threadIdx.x & (WAVE - 1);
    for (int base = 0; base < w.len; base += WAVE)
        if (base + lane < w.len) wall_node<Fmt, EXPORT>(P, w.x0 + base + lane, src, dst, tk);
}

// ---------------------------------------------------------------------------
// step kernel: one launch per time step.  The host lays the work list out
// slot by slot (slot = block * Tuning::block_waves + wave) so that wall items
// start first and each XCD's blocks cover a few contiguous bands of rows;
// kind 2 marks an empty slot.
// ---------------------------------------------------------------------------

// One wavefront's share of one step: work item w of case P, from buffer
// `parity` into the other one; tk is the step counter of the stochastic
// rounding.  EXPORT: also write the macros of the new time level and the
// divergence flag (the last step of a call).
template <typename Fm, bool EXPORT>
__device__ __forceinline__ void step_item(const CaseParams& P, const WorkItem& w, int parity, unsigned tk,
                                          typename Fm::C* park)
{
    if (w.kind == 0) {
        const char* src = static_cast<const char*>(P.buf[parity]);
        char* dst = static_cast<char*>(P.buf[parity ^ 1]);
        bool xw = false;
        if constexpr (Tuning<Fm>::xw_strips) xw = P.wall_x && (w.x0 == P.xlo || w.x0 + STRIP_COLS >= P.nx - 1);
        if constexpr (Tuning<Fm>::xw_strips) {
            if (xw) {
                interior_item<Fm, EXPORT, true>(P, w, src, dst, park, tk);
                return;
            }
        }
        interior_item<Fm, EXPORT, false>(P, w, src, dst, park, tk);
    }
    else
        wall_item<Fm, EXPORT>(P, w, static_cast<const char*>(P.buf[parity]), static_cast<char*>(P.buf[parity ^ 1]), tk);
}

// work item `wid` of the list, through the constant address space: the case
// table and the work list are read-only during a launch, so they stay in
// scalar loads and registers, independent of the vector memory traffic of
// the DFs
__device__ __forceinline__ WorkItem load_item(const WorkItem* work, int wid)
{
    const __attribute__((address_space(4))) WorkItem* wk = (const __attribute__((address_space(4))) WorkItem*)work + wid;
    WorkItem w;
    w.case_id = wk->case_id;
    w.kind = wk->kind;
    w.x0 = wk->x0;
    w.y0 = wk->y0;
    w.len = wk->len;
    w.dir = wk->dir;
    return w;
}
__device__ __forceinline__ const CaseParams& case_of(const CaseParams* cases, int k)
{
    return *(const CaseParams*)(((const __attribute__((address_space(4))) CaseParams*)cases) + k);
}

template <typename Fm, bool EXPORT>
__global__ __launch_bounds__(WAVE * Tuning<Fm>::block_waves)
__attribute__((amdgpu_waves_per_eu(Tuning<Fm>::waves, 8))) void step_kernel(
    const CaseParams* __restrict__ cases, const WorkItem* __restrict__ work, int nwork, int parity)
{
    const int wid = __builtin_amdgcn_readfirstlane(blockIdx.x * Tuning<Fm>::block_waves + (threadIdx.x >> 6));
    if (wid >= nwork) return;
    const WorkItem w = load_item(work, wid);
    if (w.kind == 2) return;
    progress_priority<Fm>(0, 1);
    const CaseParams& P = case_of(cases, w.case_id);
    // step counter of the stochastic rounding: every wavefront of the case
    // reads this step's value and writes the next step's (the same value)
    unsigned tk = 0u;
    if constexpr (sr::used<Fm>) {
        tk = __builtin_amdgcn_readfirstlane(*as_global<unsigned>(P.tick + parity));
        if ((threadIdx.x & (WAVE - 1)) == 0) *as_global_mut<unsigned>(P.tick + (parity ^ 1)) = tk + 1u;
    }
    using C = typename Fm::C;
    __shared__ C park_lds[Tuning<Fm>::park ? Tuning<Fm>::block_waves * 18 * WAVE : 1];
    C* park = park_lds + (Tuning<Fm>::park ? (threadIdx.x >> 6) * 18 * WAVE : 0);
    step_item<Fm, EXPORT>(P, w, parity, tk, park);
}

// ---------------------------------------------------------------------------
// persistent kernel: n steps in one launch.  Every wavefront keeps its work
// item for all n steps.  Between two steps the waves of a block meet at a
// barrier, and then one of them (the block's first wavefront with an item)
// arrives, once for each case among the block's items, at that case's
// counter and waits until every block holding the case has arrived (release
// and acquire at device scope), so the cases of a batch advance
// independently and no launch boundary separates the steps.  The host
// launches it only if every block is resident at once (checked against the
// kernel's occupancy), so every awaited block runs; every wait is bounded
// all the same: after `spin_limit` polls the waiting wavefront raises the
// abort word and every block leaves, so the kernel always ends.  In
// lockstep formats the waves of a block also meet at a barrier per row; a
// wavefront whose item is shorter than the longest one of its block
// executes the missing barriers at the end of each step, so the waves of a
// block meet the same number of barriers per step.
// ---------------------------------------------------------------------------


// The leader's part of a block's step barrier: arrive at the counters of the
// block's cases (ids[0 .. n)) and wait until each has reached `step` times
// its arrivals per step; false if the wait was abandoned.  Fence-to-fence
// synchronisation: the release fence orders the block's stores of the step
// (gathered by the block barrier before it) before the relaxed arrivals,
// and the acquire fence after the wait orders the next step's loads after
// it.  The polls themselves are relaxed: an acquire load at device scope
// makes the wavefront invalidate its XCD's L2 after every poll, which costs
// every other wavefront on that XCD its cached lines.
__device__ __forceinline__ bool case_barrier(const PersistentSync& S, const int* ids, int n, unsigned step)
{
    int ok = 1;
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        for (int k = 0; k < n; ++k)
            __hip_atomic_fetch_add(S.counter + ids[k], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned polls = 0;
        for (int k = 0; k < n && ok; ++k) {
            const unsigned* cnt = S.counter + ids[k];
            const unsigned target = unsigned(S.case_arrivals[ids[k]]) * step;
            while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
                if (__hip_atomic_load(S.abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
                    ok = 0;
                    break;
                }
                if (++polls > S.spin_limit) {
                    __hip_atomic_store(S.abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ok = 0;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
    }
    // lane 0's outcome for the whole wavefront, and the acquire for the block
    ok = __builtin_amdgcn_readfirstlane(ok);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    return ok != 0;
}

template <typename Fm>
__global__ __launch_bounds__(WAVE * Tuning<Fm>::block_waves)
__attribute__((amdgpu_waves_per_eu(Tuning<Fm>::waves, 8))) void persistent_kernel(
    const CaseParams* __restrict__ cases, const WorkItem* __restrict__ work, int nwork, int parity, int nsteps,
    PersistentSync S)
{
    constexpr int PB = Tuning<Fm>::block_waves;
    const int wid = __builtin_amdgcn_readfirstlane(blockIdx.x * PB + (threadIdx.x >> 6));
    if (wid >= nwork) return;
    const WorkItem w = load_item(work, wid);
    if (w.kind == 2) return;
    // the block's items: the longest interior one (row barriers per step),
    // its first wavefront with an item (the leader) and its cases
    const int first = wid - (threadIdx.x >> 6);
    int rows_max = 0, leader = -1, ncase = 0;
    int ids[PB];
    for (int k = 0; k < PB && first + k < nwork; ++k) {
        const WorkItem o = load_item(work, first + k);
        if (o.kind == 2) continue;
        if (o.kind == 0) rows_max = max(rows_max, o.len);
        if (leader < 0) leader = first + k;
        bool seen = false;
        for (int j = 0; j < ncase; ++j) seen = seen || ids[j] == o.case_id;
        if (!seen) ids[ncase++] = o.case_id;
    }
    __shared__ int abandoned;
    const CaseParams& P = case_of(cases, w.case_id);
    unsigned tk0 = 0u;
    if constexpr (sr::used<Fm>) tk0 = __builtin_amdgcn_readfirstlane(*as_global<unsigned>(P.tick + parity));
    using C = typename Fm::C;
    __shared__ C park_lds[Tuning<Fm>::park ? PB * 18 * WAVE : 1];
    C* park = park_lds + (Tuning<Fm>::park ? (threadIdx.x >> 6) * 18 * WAVE : 0);
    for (int s = 0; s < nsteps; ++s) {
        const int par = (parity + s) & 1;
        const unsigned tk = tk0 + unsigned(s);
        progress_priority<Fm>(0, 1);
        if constexpr (sr::used<Fm>) {
            if ((threadIdx.x & (WAVE - 1)) == 0) *as_global_mut<unsigned>(P.tick + (par ^ 1)) = tk + 1u;
        }
        if (s + 1 < nsteps) step_item<Fm, false>(P, w, par, tk, park);
        else step_item<Fm, true>(P, w, par, tk, park);
        if constexpr (Tuning<Fm>::lockstep) {
            const int own = w.kind == 0 ? w.len : 0;
            for (int i = own; i < rows_max; ++i) __syncthreads();
        }
        if (s + 1 < nsteps) {
            __syncthreads();   // the block's stores of the step, gathered for the leader's release
            if (wid == leader) {
                const bool ok = case_barrier(S, ids, ncase, unsigned(s + 1));
                if ((threadIdx.x & (WAVE - 1)) == 0) abandoned = ok ? 0 : 1;
            }
            __syncthreads();   // the leader's acquire, passed on to the block
            if (abandoned) return;
        }
    }
}

// ---------------------------------------------------------------------------
// initial state (t = 0): m = m^eq - F_m/2, n = n^eq - Q_m/2 at every node,
// collided with gradients of the initial fields, written post-collision into
// the current source buffer (with ghost cells) and exported
// ---------------------------------------------------------------------------
template <typename C>
__device__ __forceinline__ double init_state(const CaseParams& P, const Coef<C>& K, const double* fld, int x, int y,
                                             NodeState<C>& s)
{
    const long long nn = (long long)P.nx * P.ny;
    const long long i = (long long)y * P.nx + x;
    return state_prescribed<C>(K, P.eos, fld[i], fld[nn + i], fld[2 * nn + i], fld[3 * nn + i], s);
}

template <typename C>
__device__ __forceinline__ void init_rho_p(const CaseParams& P, const Coef<C>& K, const double* fld, int x, int y,
                                           C& rho, C& p)
{
    const int xw = wrap_axis(x, P.nx, P.wall_x), yw = wrap_axis(y, P.ny, P.wall_y);
    const long long nn = (long long)P.nx * P.ny;
    const long long i = (long long)yw * P.nx + xw;
    rho = C(fld[i] - K.rho0_d);
    p = C(eos_pressure_d<C>(K, P.eos, fld[i], fld[3 * nn + i]) - K.p0_d);
}

template <typename Fmt>
__global__ __launch_bounds__(256) void init_kernel(const CaseParams* __restrict__ cases, int case_id,
                                                   const double* __restrict__ fld, int parity, unsigned t0)
{
    using C = typename Fmt::C;
    const CaseParams& P = cases[case_id];
    const Coef<C>& K = coef<C>(P);
    const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid == 0) P.tick[parity] = t0;   // step counter of the stochastic rounding
    if (gid >= (long long)P.nx * P.ny) return;
    const int x = int(gid % P.nx), y = int(gid / P.nx);
    NodeState<C> s;
    const double T_d = init_state<C>(P, K, fld, x, y, s);
    const int sx = side_x(P, x), sy = side_y(P, y);
    C gr[2], gp[2];
    if (sx < 0 && sy < 0) {
        C sr[2] = {C(0), C(0)}, spp[2] = {C(0), C(0)};
#pragma unroll
        for (int q = 1; q < 9; ++q) {
            C r, p;
            init_rho_p<C>(P, K, fld, x + EXq(q), y + EYq(q), r, p);
            const C wq = (q <= 4) ? C(1.0 / 3.0) : C(1.0 / 12.0);   // 3 w_q
            sr[0] += wq * C(EXq(q)) * r;
            sr[1] += wq * C(EYq(q)) * r;
            spp[0] += wq * C(EXq(q)) * p;
            spp[1] += wq * C(EYq(q)) * p;
        }
        gr[0] = sr[0]; gr[1] = sr[1]; gp[0] = spp[0]; gp[1] = spp[1];
    } else {
#pragma unroll
        for (int ax = 0; ax < 2; ++ax) {
            const int dx = ax == 0 ? 1 : 0, dy = ax == 0 ? 0 : 1;
            const int sd = ax == 0 ? sx : sy;
            C r1, p1, r2, p2;
            if (sd == 0 || sd == 2) {
                init_rho_p<C>(P, K, fld, x + dx, y + dy, r1, p1);
                init_rho_p<C>(P, K, fld, x + 2 * dx, y + 2 * dy, r2, p2);
                gr[ax] = (C(-3) * s.drho + C(4) * r1 - r2) * C(0.5);
                gp[ax] = (C(-3) * s.dp + C(4) * p1 - p2) * C(0.5);
            } else if (sd == 1 || sd == 3) {
                init_rho_p<C>(P, K, fld, x - dx, y - dy, r1, p1);
                init_rho_p<C>(P, K, fld, x - 2 * dx, y - 2 * dy, r2, p2);
                gr[ax] = (C(3) * s.drho - C(4) * r1 + r2) * C(0.5);
                gp[ax] = (C(3) * s.dp - C(4) * p1 + p2) * C(0.5);
            } else {
                init_rho_p<C>(P, K, fld, x + dx, y + dy, r1, p1);
                init_rho_p<C>(P, K, fld, x - dx, y - dy, r2, p2);
                gr[ax] = (r1 - r2) * C(0.5);
                gp[ax] = (p1 - p2) * C(0.5);
            }
        }
    }
    Rates<C> r;
    local_rates<C>(K, P.visc_law, s, r);
    const Forcing<C> F = forcing<C>(K, P.per_mass, s);
    C meq[9], Fm[9], neq[9], Qm[9], Z[9], mb[9], nb[9], fb[9], gb[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) Z[q] = C(0);
    meq_f<C>(s, meq);
    force_moments<C>(s, F, Fm);
    neq_g<C>(K, s, neq);
    source_moments<C>(s, F, Qm);
    post_collision<C>(s, r, P.cubic, meq, Fm, Z, Z, neq, Qm, Z, Z, gr[0], gr[1], gp[0], gp[1], mb, nb);
    from_moments<C>(mb, fb);
    from_moments<C>(nb, gb);
    char* dst = static_cast<char*>(P.buf[parity]);
    store_node<Fmt>(P, dst, x, y, fb, gb, t0);
    if (sx >= 0 || sy >= 0) store_ghosts<Fmt>(P, dst, x, y, fb, gb, t0);
    export_node<C>(P, x, y, s, T_d);
}

// ---------------------------------------------------------------------------
// launchers of one storage format (instantiated per format)
// ---------------------------------------------------------------------------
template <typename Fm>
int launch_step_v(const CaseParams* d_cases, const WorkItem* d_work, int nwork, int parity, int export_macros,
                  hipStream_t stream)
{
    constexpr int pb = Tuning<Fm>::block_waves;
    const dim3 block(WAVE * pb);
    const dim3 grid((nwork + pb - 1) / pb);
    if (export_macros)
        hipLaunchKernelGGL((step_kernel<Fm, true>), grid, block, 0, stream, d_cases, d_work, nwork, parity);
    else
        hipLaunchKernelGGL((step_kernel<Fm, false>), grid, block, 0, stream, d_cases, d_work, nwork, parity);
    return int(hipGetLastError());
}

template <typename Fm>
int launch_persistent_v(const CaseParams* d_cases, const WorkItem* d_work, int nwork, int parity, int nsteps,
                        const PersistentSync& sync, hipStream_t stream)
{
    constexpr int pb = Tuning<Fm>::block_waves;
    const dim3 block(WAVE * pb);
    const dim3 grid((nwork + pb - 1) / pb);
    hipLaunchKernelGGL((persistent_kernel<Fm>), grid, block, 0, stream, d_cases, d_work, nwork, parity, nsteps, sync);
    return int(hipGetLastError());
}

// resident blocks per CU of the persistent kernel
template <typename Fm>
int persistent_blocks_v(int* blocks_per_cu)
{
    *blocks_per_cu = 0;
    return int(hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, persistent_kernel<Fm>,
                                                            WAVE * Tuning<Fm>::block_waves, 0));
}

template <typename Fm>
int step_shape_v(StepShape* out)
{
    out->lockstep = Tuning<Fm>::lockstep ? 1 : 0;
    out->xw_strips = Tuning<Fm>::xw_strips ? 1 : 0;
    out->block_waves = Tuning<Fm>::block_waves;
    out->xw_cost = Tuning<Fm>::xw_cost;
    int n = 0;
    const hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_kernel<Fm, false>,
                                                                      WAVE * Tuning<Fm>::block_waves, 0);
    out->blocks_per_cu = e == hipSuccess ? n : 0;
    return int(e);
}

// Calls fn with Variant<Base, v> for a variant index v in [0, NUM_STEP_VARIANTS).
template <typename Base, typename Fn>
int with_variant(int v, Fn&& fn)
{
    switch (v) {
    case 1: return fn(Variant<Base, 1>{});
    case 2: return fn(Variant<Base, 2>{});
    case 3: return fn(Variant<Base, 3>{});
    case 4: return fn(Variant<Base, 4>{});
    default: return fn(Variant<Base, 0>{});
    }
}

template <typename Base>
int launch_step_fmt(int variant, const CaseParams* d_cases, const WorkItem* d_work, int nwork, int parity,
                    int export_macros, hipStream_t stream)
{
    if (nwork == 0) return 0;
    return with_variant<Base>(variant, [&](auto fm) {
        return launch_step_v<decltype(fm)>(d_cases, d_work, nwork, parity, export_macros, stream);
    });
}

template <typename Base>
int step_shape_fmt(int variant, StepShape* out)
{
    return with_variant<Base>(variant, [&](auto fm) { return step_shape_v<decltype(fm)>(out); });
}

template <typename Base>
int launch_persistent_fmt(int variant, const CaseParams* d_cases, const WorkItem* d_work, int nwork, int parity,
                          int nsteps, const PersistentSync& sync, hipStream_t stream)
{
    if (nwork == 0 || nsteps <= 0) return 0;
    return with_variant<Base>(variant, [&](auto fm) {
        return launch_persistent_v<decltype(fm)>(d_cases, d_work, nwork, parity, nsteps, sync, stream);
    });
}

template <typename Base>
int persistent_blocks_fmt(int variant, int* blocks_per_cu)
{
    return with_variant<Base>(variant, [&](auto fm) { return persistent_blocks_v<decltype(fm)>(blocks_per_cu); });
}

template <typename Base>
int launch_init_fmt(const CaseParams* d_cases, int case_id, long long nodes, const double* d_fields, int parity,
                    unsigned t0, hipStream_t stream)
{
    const dim3 grid(unsigned((nodes + 255) / 256)), block(256);
    hipLaunchKernelGGL((init_kernel<Base>), grid, block, 0, stream, d_cases, case_id, d_fields, parity, t0);
    return int(hipGetLastError());
}

// One translation unit per format defines its entry points with this macro.
#define LBM_DEFINE_FORMAT(NAME, FMT)                                                                         \
    int launch_step_##NAME(int variant, const CaseParams* d_cases, const WorkItem* d_work, int nwork,        \
                           int parity, int export_macros, hipStream_t stream)                                \
    {                                                                                                        \
        return launch_step_fmt<FMT>(variant, d_cases, d_work, nwork, parity, export_macros, stream);         \
    }                                                                                                        \
    int step_shape_##NAME(int variant, StepShape* out) { return step_shape_fmt<FMT>(variant, out); }         \
    int launch_persistent_##NAME(int variant, const CaseParams* d_cases, const WorkItem* d_work, int nwork,  \
                                 int parity, int nsteps, const PersistentSync& sync, hipStream_t stream)     \
    {                                                                                                        \
        return launch_persistent_fmt<FMT>(variant, d_cases, d_work, nwork, parity, nsteps, sync, stream);    \
    }                                                                                                        \
    int persistent_blocks_##NAME(int variant, int* blocks_per_cu)                                            \
    {                                                                                                        \
        return persistent_blocks_fmt<FMT>(variant, blocks_per_cu);                                           \
    }                                                                                                        \
    int launch_init_##NAME(const CaseParams* d_cases, int case_id, long long nodes, const double* d_fields,  \
                           int parity, unsigned t0, hipStream_t stream)                                      \
    {                                                                                                        \
        return launch_init_fmt<FMT>(d_cases, case_id, nodes, d_fields, parity, t0, stream);                  \
    }

}  // namespace lbm

