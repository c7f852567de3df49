// Index arithmetic of the 4^4-block SAP half-sweep (tm_sap.hip), in host- and
// device-callable form so that it can be checked exhaustively on the CPU.
//
// Workgroup j of a half-sweep of colour c owns the j-th Schwarz block of that
// colour (blocks are coloured by the parity of the sum of their coordinates,
// section 2.4), with the block coordinate along x (the fastest axis) chosen to
// give the colour.  Thread l owns the site with local coordinates
// (l>>6, (l>>4)&3, (l>>2)&3, l&3) in (t, z, y, x).  Each wave w also stages one
// face layer of the halo: lane p (0..63) of wave w loads the site just above the
// block's upper face on array axis w and the one just below its lower face, at
// face position p (the lexicographic index over the other three axes).
#pragma once

#include "tm_device.h"

namespace tmsap {

struct S44Site {
    int B[4];          // block coordinates (array axes t, z, y, x)
    long long blk;     // block index (lexicographic over the block grid)
    long long s;       // the thread's site in the tiled layout
    int L[4];          // local coordinates
    bool fin[4], bin[4];  // the +mu / -mu neighbour lies inside the block (mu = t, x, y, z)
    int str[4];        // local-index stride of direction mu
    int fsrc[4];       // forward source: local index (fin) or upper-halo entry axis*64 + position
    int bsrc[4];       // backward source: local index (bin) or lower-halo entry axis*64 + position
    int bcol[4];       // backward source inside the block: local index (bin) or, for a lower-face
                       // site, the upper-face site of its column, whose product slot holds the halo
    int parity;        // (t + z + y + x) mod 2 of the global coordinates
    // halo duty of the thread: array axis wax (= wave), face position hp (= lane)
    int wax, wmu, hp;
    int top;           // local index of the upper-face site (on axis wax) of position hp's column
    long long up_site, dn_site;  // sites just above / below the block on axis wax at position hp
    bool up_wrap, dn_wrap;       // those hops cross the lattice boundary
};

// Block coordinates of workgroup j in the half-sweep of `colour` (g.nb[3] even).
__host__ __device__ inline void s44_block(const Geo& g, int colour, long long j, int B[4]) {
    const int half3 = g.nb[3] >> 1;
    const int k3 = (int)(j % half3);
    j /= half3;
    B[2] = (int)(j % g.nb[2]);
    j /= g.nb[2];
    B[1] = (int)(j % g.nb[1]);
    B[0] = (int)(j / g.nb[1]);
    B[3] = 2 * k3 + ((colour + B[0] + B[1] + B[2]) & 1);
}

// Tiled-layout index of global coordinates c on 4^4 tiles (shifts and masks;
// the general coords_site divides by the tile extents).
__host__ __device__ inline long long s44_site_of(const Geo& g, const int c[4]) {
    const long long blk = (((long long)(c[0] >> 2) * g.nb[1] + (c[1] >> 2)) * g.nb[2] + (c[2] >> 2)) * g.nb[3] + (c[3] >> 2);
    return blk * 256 + (((c[0] & 3) * 4 + (c[1] & 3)) * 4 + (c[2] & 3)) * 4 + (c[3] & 3);
}

// The thread's part of the setup, given the block coordinates B (the same for
// the whole workgroup) and its block index blk.  Every loop is unrolled and
// every array index a compile-time constant after unrolling (the run-time axis
// wax enters only through comparisons), so the struct lives in registers.
__host__ __device__ inline void s44_lane(const Geo& g, const int B[4], long long blk, int l, S44Site& t) {
#pragma unroll
    for (int a = 0; a < 4; ++a) t.B[a] = B[a];
    t.blk = blk;
    t.s = t.blk * 256 + l;
    t.L[0] = l >> 6;
    t.L[1] = (l >> 4) & 3;
    t.L[2] = (l >> 2) & 3;
    t.L[3] = l & 3;
    int csum = 0;
#pragma unroll
    for (int a = 0; a < 4; ++a) csum += t.B[a] * 4 + t.L[a];
    t.parity = csum & 1;
#pragma unroll
    for (int mu = 0; mu < 4; ++mu) {
        const int ax = axis_of(mu);
        t.str[mu] = 1 << (2 * (3 - ax));
        t.fin[mu] = t.L[ax] < 3;
        t.bin[mu] = t.L[ax] > 0;
        int p = 0;
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (q != ax) p = p * 4 + t.L[q];
        t.fsrc[mu] = t.fin[mu] ? l + t.str[mu] : ax * 64 + p;
        t.bsrc[mu] = t.bin[mu] ? l - t.str[mu] : ax * 64 + p;
        t.bcol[mu] = t.bin[mu] ? l - t.str[mu] : l + 3 * t.str[mu];
    }
    t.wax = l >> 6;
    t.wmu = t.wax == 0 ? 0 : 4 - t.wax;
    t.hp = l & 63;
    // face position hp: lexicographic over the axes other than wax, the last one fastest
    int up[4], dn[4];
    int p = t.hp;
    t.top = 0;
#pragma unroll
    for (int q = 3; q >= 0; --q) {
        const bool on = q == t.wax;
        up[q] = on ? 0 : (p & 3);
        p = on ? p : p >> 2;
        t.top += (on ? 3 : up[q]) << (2 * (3 - q));
    }
    t.up_wrap = false;
    t.dn_wrap = false;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const bool on = q == t.wax;
        const int base = t.B[q] * 4;
        int u = on ? base + 4 : base + up[q];
        int d = on ? base - 1 : base + up[q];
        if (on && u >= g.d[q]) {
            u -= g.d[q];
            t.up_wrap = true;
        }
        if (on && d < 0) {
            d += g.d[q];
            t.dn_wrap = true;
        }
        up[q] = u;
        dn[q] = d;
    }
    t.up_site = s44_site_of(g, up);
    t.dn_site = s44_site_of(g, dn);
}

// Block index of block coordinates B.
__host__ __device__ inline long long s44_block_index(const Geo& g, const int B[4]) {
    return (((long long)B[0] * g.nb[1] + B[1]) * g.nb[2] + B[2]) * g.nb[3] + B[3];
}

__host__ __device__ inline void s44_setup(const Geo& g, int colour, long long j, int l, S44Site& t) {
    int B[4];
    s44_block(g, colour, j, B);
    s44_lane(g, B, s44_block_index(g, B), l, t);
}

}  // namespace tmsap
