// Tile classes of a lattice sweep and the block -> tile map of the launch
// over the ring of wall tiles.  Plain C++ with host/device qualifiers only, so
// that the host-side test of the map compiles it with a CPU compiler too.
#pragma once

#if defined(__HIPCC__)
#define DK_HD __host__ __device__
#else
#define DK_HD
#endif

namespace dk {

// A tile (cells i0..i0+TX-1, j0..j0+TY-1) is of the fast kind when the grid is
// uniform and its 2-cell halo needs no wall treatment: periodic along an
// axis, or at least two cells clear of both walls of that axis.
DK_HD inline bool tile_fast(bool uniform, bool perx, bool pery, int nx, int ny, int i0, int j0, int TX, int TY)
{
    return uniform && (perx || (i0 >= 2 && i0 + TX <= nx - 2)) && (pery || (j0 >= 2 && j0 + TY <= ny - 2));
}

// On a uniform grid the fast-kind tiles form the rectangle of tile columns
// [cx0, cx1) by tile rows [ry0, ry1); the general kind is the ring around it
// (the tiles within two cells of a wall).  With on = 1 a general launch has
// one block per ring tile: the rows below the rectangle, then the side tiles
// of its rows, then the rows above, ng tiles in all.
struct Ring {
    int on, gx, cx0, cx1, ry0, ry1, ng;
};

// The ring of general tiles (on = 0 where every tile is general, or none is).
// Mirrors tile_fast per tile column and tile row.
DK_HD inline Ring ring_make(bool uniform, bool perx, bool pery, int nx, int ny, int TX, int TY)
{
    Ring r{0, 0, 0, 0, 0, 0, 0};
    const int gx = (nx + TX - 1) / TX, gy = (ny + TY - 1) / TY;
    if (!uniform) return r;
    int cx0 = gx, cx1 = 0, ry0 = gy, ry1 = 0;
    for (int k = 0; k < gx; k++) {
        const int i0 = k * TX;
        if (perx || (i0 >= 2 && i0 + TX <= nx - 2)) {
            cx0 = k < cx0 ? k : cx0;
            cx1 = k + 1;
        }
    }
    if (cx1 <= cx0) cx0 = cx1 = 0;
    for (int k = 0; k < gy; k++) {
        const int j0 = k * TY;
        if (pery || (j0 >= 2 && j0 + TY <= ny - 2)) {
            ry0 = k < ry0 ? k : ry0;
            ry1 = k + 1;
        }
    }
    if (ry1 <= ry0) ry0 = ry1 = 0;
    const long long nfast = (long long)(cx1 - cx0) * (ry1 - ry0);
    if (nfast == 0) return r;
    r = Ring{1, gx, cx0, cx1, ry0, ry1, (int)((long long)gx * gy - nfast)};
    return r;
}

// Tile of block b of a ring launch.  XCD-aware: blocks are dealt to the nxcd
// XCDs round-robin, and the blocks of one XCD take a contiguous run of ring
// tiles.
DK_HD inline void ring_tile_of(const Ring &r, int nxcd, int b_in, int &tx, int &ty)
{
    const int per = r.ng / nxcd, rem = r.ng % nxcd;
    const int x = b_in % nxcd, slot = b_in / nxcd;
    const int b = x * per + (x < rem ? x : rem) + slot;
    const int fx = r.cx1 - r.cx0, side = r.gx - fx;
    const int nb = r.ry0 * r.gx, nm = (r.ry1 - r.ry0) * side;
    if (b < nb) {
        ty = b / r.gx;
        tx = b % r.gx;
    } else if (b - nb < nm) {
        const int k = b - nb, c = k % side;
        ty = r.ry0 + k / side;
        tx = c < r.cx0 ? c : c + fx;
    } else {
        const int k = b - nb - nm;
        ty = r.ry1 + k / r.gx;
        tx = k % r.gx;
    }
}

}  // namespace dk
