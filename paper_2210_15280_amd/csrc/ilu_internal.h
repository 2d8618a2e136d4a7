// Internal definitions shared by the host code and the HIP kernels of libilu.
//
// Lattice of one macro-tetrahedron (Sec. 2.1): interior points (x,y,z) with
// x,y,z >= 1 and x+y+z <= n-1, n = 2^L.  The kernels work in the skewed
// coordinates
//     u = x + y + z,   v = y + z,   w = z,
// in which all seven lower stencil offsets of D_l have non-negative
// components, and the hyperplane index of the wavefront schedule is
//     t = x + 2y + 3z = u + v + w.
// A "row" is a fixed (v, w), i.e. a fixed (y, z); it runs along x (= along u).
// Rows are tiled into BV x BW blocks in (v, w) (BV, BW multiples of 8); one
// workgroup owns one block.  Lanes go by 8x8 tiles of rows: each 64-lane
// group (one wavefront) holds one tile (lane_rc / lane_at), so the rows a
// wavefront shares are close in both v and w and their hyperplane windows
// overlap as much as possible.
//
// Stream layout.  Every per-point array (x, b, r, w, stencil and factor
// arrays) is stored block by block; inside a block the element of lane l at
// hyperplane t sits at  base + (t - tlo) * LPB + l, LPB = BV*BW lanes per
// block.  A lane's row pointer is rp = base - tlo * LPB + l, so point
// (row, t) lives at rp + LPB t.  At a fixed t the lanes of a block are
// contiguous: every wavefront access of the sweep kernels is one coalesced
// 512 B (FP64) or 256 B (FP32) transaction.  Block windows
// are padded by PAD zero steps on both sides so that neighbour reads of
// interior points never leave their block; rows outside the lattice point to
// the zero region at the start of every stream.
#pragma once

#include <stdint.h>

namespace ilu {

constexpr int WAVE = 64;    // wavefront size; point kernels handle 64-lane groups
constexpr int PAD = 2;      // zero steps on each side of a block window
constexpr int TAIL = 4;     // zero steps after the last block (unconditional neighbour loads)
constexpr int NDIR = 15;
constexpr int NLOW = 7;

// Lane row-pointer slots: own row and the six neighbour rows in (v, w).
enum RowSlot { R_SELF = 0, R_VM = 1, R_WM = 2, R_VMWM = 3, R_VP = 4, R_WP = 5, R_VPWP = 6 };

struct TetDev {
    int32_t level, n, kind, stride;
    double v0[3];        // base vertex v1
    double J[9];         // J[3*r + c]: column c = d_{c+1} = v_{c+2} - v1
    double cp[4];        // coefficient parameters
    int64_t lex_off;     // offset of this tet in user vectors
    int64_t N;           // interior points
    int32_t blk0, nblk;  // block range in the global block table
    int32_t deg[3];      // surrogate degrees
    int32_t ncoef;       // (dg_x+1)(dg_y+1)(dg_z+1)
    int32_t samp_M[8];   // sample simplex side per fitted direction (0..6 lower, 7 = c)
    int64_t samp_off[8]; // offset of each direction's samples in the sample buffer
    int64_t samp_cnt[8];
};

struct BlockDev {
    int32_t tet, V0, W0;
    int32_t tb, te;      // first / last hyperplane with an active lane
    int32_t tlo;         // tb - PAD: time origin of the block's storage
    int32_t len;         // te - tb + 1 + 2 PAD stored steps
    int32_t pred[3];     // forward-sweep predecessors: (V-1,W), (V,W-1), (V-1,W-1); -1 if none
    int32_t succ[3];     // backward-sweep predecessors: (V+1,W), (V,W+1), (V+1,W+1)
    int32_t edge;        // some row with y <= 2 or z == 1 (variant V1: streamed factors)
    int64_t base;        // stream index of (tlo, lane 0)
    int64_t xoff;        // first entry of the block's exchange window: len x (BV + BW) entries
};

// Row (vl, wl) = (v - V0, w - W0) of lane l in a block of width bv, and back:
// 64-lane group g holds the 8x8 tile (g mod (bv/8), g div (bv/8)) of the
// block, row-major inside the tile.
__host__ __device__ inline void lane_rc(int l, int bv, int* vl, int* wl) {
    const int g = l >> 6, r = l & 63, gv = bv >> 3;
    *vl = (g % gv) * 8 + (r & 7);
    *wl = (g / gv) * 8 + (r >> 3);
}
__host__ __device__ inline int lane_at(int vl, int wl, int bv) {
    return (((wl >> 3) * (bv >> 3) + (vl >> 3)) << 6) + ((wl & 7) << 3) + (vl & 7);
}

// Lane-group decoding for the point-parallel kernels: workgroup x-index g
// covers lanes [64 (g % groups), +64) of block g / groups.

struct LaneDev {
    int64_t rp[7];       // row pointers, RowSlot order; zero-region pointer if the row is outside
    int32_t v, w;        // row coordinates; v = 0 marks an unused lane
    int32_t v1f[4];      // variant V1: first set-F index of the rows R_SELF, R_VP, R_WP, R_VPWP
    int32_t v1b;         // variant V1: first set-B index of the own row (-1: row outside)
    int32_t gt[2];       // hyperplanes [gt[0], gt[1]] with an active point in this lane's 64-lane
                         // group (empty if gt[0] > gt[1]): the point-parallel kernels skip the rest
    int32_t gl[7];       // global lane (block * lanes per block + lane) of the own row and the six
                         // neighbour rows, RowSlot order; -1 if the row is outside (the setup's
                         // hyperplane ring is indexed by it)
    int32_t pad_[2];
};

// Point sets of variant V1 (Sec. 4.1), per row (y, z) with xmax = n-1-y-z:
//   F, the boundary points: interior points with a stencil neighbour on the
//      macro boundary, i.e. min(x, y, z) = 1 or x = xmax.  Their exact factors
//      L^p_d and 1/D^p are stored.
//   B, the points whose backward substitution may need a stored factor: F and
//      every point with an upper neighbour p - d in F, which adds x = 2,
//      y = 2 and x = xmax - 1 (upper offsets have dz >= 0, so no z = 2).
// Rows with y == 1 or z == 1 lie wholly in F, rows with y <= 2 or z == 1
// wholly in B; any other row holds x in {1, xmax} of F and x in
// {1, 2, xmax-1, xmax} of B.  Points of a set are numbered row by row, x
// ascending; *_pos is the position of x inside its row's run (-1: not in the set).
__host__ __device__ inline bool v1f_whole(int y, int z) { return y == 1 || z == 1; }
__host__ __device__ inline bool v1b_whole(int y, int z) { return y <= 2 || z == 1; }
__host__ __device__ inline int v1f_count(int xmax, int y, int z) {
    return xmax < 1 ? 0 : v1f_whole(y, z) ? xmax : (xmax < 2 ? xmax : 2);
}
__host__ __device__ inline int v1b_count(int xmax, int y, int z) {
    return xmax < 1 ? 0 : v1b_whole(y, z) ? xmax : (xmax < 4 ? xmax : 4);
}
__host__ __device__ inline int v1f_pos(int x, int xmax, int y, int z) {
    if (v1f_whole(y, z)) return x - 1;
    if (x == 1) return 0;
    if (x == xmax) return 1;
    return -1;
}
__host__ __device__ inline int v1b_pos(int x, int xmax, int y, int z) {
    if (v1b_whole(y, z) || xmax <= 4 || x <= 2) return x - 1;
    if (x >= xmax - 1) return x - xmax + 3;
    return -1;
}
// The same positions as selects only (no branches for the compiler to keep):
// the sweep kernels evaluate them per lane on every hyperplane.
__host__ __device__ inline int v1f_pos_sel(int x, int xmax, int y, int z) {
    const bool whole = (y == 1) | (z == 1);
    int p = x == xmax ? 1 : -1;
    p = x == 1 ? 0 : p;
    return whole ? x - 1 : p;
}
__host__ __device__ inline int v1b_pos_sel(int x, int xmax, int y, int z) {
    const bool low = (y <= 2) | (z == 1) | (xmax <= 4) | (x <= 2);
    const int p = x >= xmax - 1 ? x - xmax + 3 : -1;
    return low ? x - 1 : p;
}

// Dataflow exchange buffer: word index of entry j (0 <= j < nx = BV + BW) at
// hyperplane t of the block whose window starts at entry xoff and whose
// storage time origin is tlo; wds 64-bit words per entry.  Used by the sweep
// kernels and by the host-side layout replay alike.
__host__ __device__ inline int64_t xch_word(int64_t xoff, int tlo, int nx, int wds, int t, int j) {
    return (xoff + (int64_t)(t - tlo) * nx + j) * wds;
}

// Producer lane (vl, wl) of outgoing exchange entry j (0 <= j < BV + BW) in
// sweep direction dir (0 = forward, 1 = backward): j < BW is the column entry
// of row wl = j on the last column in sweep direction, j >= BW the row entry
// of column vl = j - BW on the last row.  The corner lane appears in both.
__host__ __device__ inline void xch_out_lane(int dir, int j, int bv, int bw, int* vl, int* wl) {
    if (j < bw) { *vl = dir == 0 ? bv - 1 : 0; *wl = j; }
    else { *vl = j - bw; *wl = dir == 0 ? bw - 1 : 0; }
}
// Incoming halo role of thread l: k = producer slot (0: column neighbour,
// 1: row neighbour, 2: corner; pred[k] forward, succ[k] backward) and the
// producer's entry j.  Returns false for threads without a role.
__host__ __device__ inline bool xch_halo_role(int dir, int l, int bv, int bw, int* k, int* j) {
    if (l < bw) { *k = 0; *j = l; return true; }
    if (l < bw + bv) { *k = 1; *j = l; return true; }
    if (l == bw + bv) { *k = 2; *j = dir == 0 ? bw + bv - 1 : bw; return true; }
    return false;
}

// Fitted directions: 0..6 = lower directions of D_l, 7 = centre (fits 1/D).
constexpr int NFIT = 8;

}  // namespace ilu
