// Staging geometry of the LDS-staged residual (k_residual_lds): which LDS cell
// of a hyperplane slice holds which row, and which lane loads each halo row.
// Host and device code share these functions, so the host layout check replays
// the kernel's own indices.
#pragma once

#include "kernels_common.h"

namespace ilu {

constexpr int RL_P = 4;  // slices a workgroup keeps in flight (registers)

template <int BV, int BW>
struct RlGeo {
    static constexpr int NT = BV * BW;
    static constexpr int XH = 2 * BV + 2 * BW + 2;  // x halo cells
    static constexpr int AH = 4 * BW + 4 * BV + 2;  // stencil values at the upper halo rows
    static constexpr int XC = NT + XH;              // x cells of a slice
    static constexpr int AC = 6 * NT + AH;          // stencil cells of a slice (arrays 2..7)
    static constexpr int RX = 7, RA = 4;            // ring slots of x and the stencil arrays
    static constexpr int NH = XH + AH;              // halo loads per slice
    static constexpr int HJ = (NH + NT - 1) / NT;
    static constexpr int LDS = RX * XC + RA * AC;   // doubles
};

// x cell of the extended tile (cv, cw) in [-1, BV] x [-1, BW] (the corners
// (-1, BW) and (BV, -1) are never read): block rows by lane, then the halo
// sides v - 1, v + 1, w - 1, w + 1 and the corners (-1, -1), (BV, BW).
template <int BV, int BW>
__host__ __device__ inline int rl_xcell(int cv, int cw) {
    constexpr int NT = BV * BW;
    if (cv >= 0 && cv < BV && cw >= 0 && cw < BW) return lane_at(cv, cw, BV);
    if (cw >= 0 && cw < BW) return NT + (cv < 0 ? 0 : BW) + cw;
    if (cv >= 0 && cv < BV) return NT + 2 * BW + (cw < 0 ? 0 : BV) + cv;
    return NT + 2 * BW + 2 * BV + (cv < 0 ? 0 : 1);
}

// Cell of the stencil value of array a = 1 + s (s >= 1 a lower direction) at
// the upper neighbour cell (cv, cw) of a block row: the block's rows hold
// arrays 2..7, the halo rows the upper weights that the block's edge rows read
// there (arrays 2, 3, 6, 7 at the v + 1 side, 4, 5, 6, 7 at the w + 1 side, 6, 7
// at the corner).  Arrays 0 and 1 are read by their own row only.
template <int BV, int BW>
__host__ __device__ inline int rl_acell(int cv, int cw, int a) {
    constexpr int NT = BV * BW;
    if (cv < BV && cw < BW) return (a - 2) * NT + lane_at(cv, cw, BV);
    if (cv == BV && cw < BW) return 6 * NT + cw * 4 + (a < 4 ? a - 2 : a - 4);
    if (cw == BW && cv < BV) return 6 * NT + 4 * BW + cv * 4 + (a - 4);
    return 6 * NT + 4 * BW + 4 * BV + (a - 6);
}

// Halo load j of a slice (j < NH): the edge lane src whose row pointer slot
// names the halo row, the LDS cell it fills and the array (-1: x).
struct RlHalo {
    int src, slot, dst, arr;
};
template <int BV, int BW>
__host__ __device__ inline RlHalo rl_halo(int j) {
    using G = RlGeo<BV, BW>;
    constexpr int NT = G::NT;
    RlHalo o{0, R_SELF, -1, -1};
    if (j < G::XH) {
        const int h = j;
        if (h < BW) o = {lane_at(0, h, BV), R_VM, 0, -1};
        else if (h < 2 * BW) o = {lane_at(BV - 1, h - BW, BV), R_VP, 0, -1};
        else if (h < 2 * BW + BV) o = {lane_at(h - 2 * BW, 0, BV), R_WM, 0, -1};
        else if (h < 2 * BW + 2 * BV) o = {lane_at(h - 2 * BW - BV, BW - 1, BV), R_WP, 0, -1};
        else if (h == 2 * BW + 2 * BV) o = {lane_at(0, 0, BV), R_VMWM, 0, -1};
        else o = {lane_at(BV - 1, BW - 1, BV), R_VPWP, 0, -1};
        o.dst = NT + h;
    } else if (j < G::NH) {
        const int h = j - G::XH;
        if (h < 4 * BW) o = {lane_at(BV - 1, h / 4, BV), R_VP, 0, (h & 3) < 2 ? 2 + (h & 3) : 4 + (h & 3)};
        else if (h < 4 * BW + 4 * BV) o = {lane_at((h - 4 * BW) / 4, BW - 1, BV), R_WP, 0, 4 + ((h - 4 * BW) & 3)};
        else o = {lane_at(BV - 1, BW - 1, BV), R_VPWP, 0, 6 + (h - 4 * BW - 4 * BV)};
        o.dst = 6 * NT + h;
    }
    return o;
}

// Row offset (dv, dw) of a row-pointer slot.
__host__ __device__ constexpr int rl_slot_dv(int slot) {
    return (slot == R_VM || slot == R_VMWM) ? -1 : (slot == R_VP || slot == R_VPWP) ? 1 : 0;
}
__host__ __device__ constexpr int rl_slot_dw(int slot) {
    return (slot == R_WM || slot == R_VMWM) ? -1 : (slot == R_WP || slot == R_VPWP) ? 1 : 0;
}

// Activity of row (v, w) of a level with n intervals per edge: the point at
// hyperplane T is interior iff T - off lies in [1, xmax], with off = 2v + w and
// xmax = n - 1 - v for a lattice row, 0 (never) for a row outside the lattice.
// The stream slots of other (row, T) pairs hold zero.
struct RlRow {
    int off, xmax;
};
__host__ __device__ inline RlRow rl_row(int n, int v, int w) {
    const bool in = v >= 2 && v <= n - 2 && w >= 1 && w <= v - 1;
    return RlRow{2 * v + w, in ? n - 1 - v : 0};
}
__host__ __device__ inline bool rl_active(const RlRow& r, int T) {
    const int xx = T - r.off;
    return xx >= 1 && xx <= r.xmax;
}

// LDS cells of the neighbours of block row (vl, wl) in lower direction s: x at
// the lower and the upper neighbour, and (s >= 1) the upper neighbour's weight
// (array 1 + s).
template <int BV, int BW>
__host__ __device__ inline void rl_cells(int vl, int wl, int s, int* xl, int* xu, int* au) {
    const int lr = low_row(s), ur = up_row(s);
    const int dlv = (lr == R_VM || lr == R_VMWM) ? -1 : 0, dlw = (lr == R_WM || lr == R_VMWM) ? -1 : 0;
    const int duv = (ur == R_VP || ur == R_VPWP) ? 1 : 0, duw = (ur == R_WP || ur == R_VPWP) ? 1 : 0;
    *xl = rl_xcell<BV, BW>(vl + dlv, wl + dlw);
    *xu = rl_xcell<BV, BW>(vl + duv, wl + duw);
    *au = s == 0 ? -1 : rl_acell<BV, BW>(vl + duv, wl + duw, 1 + s);
}

}  // namespace ilu
