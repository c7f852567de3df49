// Exhaustive host-side check of the index arithmetic the kernels share
// (tm_device.h: site_coords, coords_site, tiled_neighbours) and of the 4^4
// SAP kernel's per-thread setup (tm_sap_index.h), against plain coordinate
// arithmetic written here: lexicographic coordinates, periodic wrap, block
// coordinates and colours.  Built for the host only and run on the CPU by
// tests/test_host_index.py; prints one line per geometry and "ALL OK".
#include <cstdio>
#include <cstdlib>
#include <set>
#include <vector>

#include "../paper_1610_02370_amd/csrc/tm_sap_index.h"

using namespace tmsap;

static int failures = 0;
#define CHECK(cond, ...)                         \
    do {                                         \
        if (!(cond)) {                           \
            if (failures < 20) {                 \
                std::printf("FAIL: " __VA_ARGS__); \
                std::printf("\n");               \
            }                                    \
            ++failures;                          \
        }                                        \
    } while (0)

static Geo make(const int d[4], const int lb[4]) {
    Geo g{};
    g.V = 1;
    g.Vb = 1;
    for (int a = 0; a < 4; ++a) {
        g.d[a] = d[a];
        g.lb[a] = lb[a];
        g.nb[a] = d[a] / lb[a];
        g.V *= d[a];
        g.Vb *= lb[a];
    }
    return g;
}

// coordinates of tiled site s, from first principles
static void coords_of(const Geo& g, long long s, int c[4]) {
    long long blk = s / g.Vb;
    int l = (int)(s % g.Vb);
    int L[4], B[4];
    L[3] = l % g.lb[3];
    L[2] = (l / g.lb[3]) % g.lb[2];
    L[1] = (l / (g.lb[3] * g.lb[2])) % g.lb[1];
    L[0] = l / (g.lb[3] * g.lb[2] * g.lb[1]);
    B[3] = (int)(blk % g.nb[3]);
    B[2] = (int)((blk / g.nb[3]) % g.nb[2]);
    B[1] = (int)((blk / ((long long)g.nb[3] * g.nb[2])) % g.nb[1]);
    B[0] = (int)(blk / ((long long)g.nb[3] * g.nb[2] * g.nb[1]));
    for (int a = 0; a < 4; ++a) c[a] = B[a] * g.lb[a] + L[a];
}

static int axis(int mu) { return mu == 0 ? 0 : 4 - mu; }  // mu = t, x, y, z -> array axes t, z, y, x

static void check_neighbours(const Geo& g) {
    std::vector<char> seen(g.V, 0);
    for (long long s = 0; s < g.V; ++s) {
        int c[4], c2[4];
        coords_of(g, s, c);
        site_coords(g, s, c2);
        for (int a = 0; a < 4; ++a) CHECK(c[a] == c2[a], "site_coords s=%lld axis %d", s, a);
        CHECK(coords_site(g, c) == s, "coords_site round trip s=%lld", s);
        CHECK(!seen[s], "site %lld twice", s);
        seen[s] = 1;
        int nf[4], nb[4], par;
        unsigned wrap;
        tiled_neighbours(g, s, nf, nb, &wrap, &par);
        CHECK(par == ((c[0] + c[1] + c[2] + c[3]) & 1), "parity s=%lld", s);
        for (int mu = 0; mu < 4; ++mu) {
            const int a = axis(mu);
            int f[4] = {c[0], c[1], c[2], c[3]}, b[4] = {c[0], c[1], c[2], c[3]};
            const bool wf = f[a] + 1 == g.d[a], wb = b[a] == 0;
            f[a] = (f[a] + 1) % g.d[a];
            b[a] = (b[a] + g.d[a] - 1) % g.d[a];
            int cf[4], cb[4];
            coords_of(g, nf[mu], cf);
            coords_of(g, nb[mu], cb);
            for (int q = 0; q < 4; ++q) {
                CHECK(cf[q] == f[q], "forward neighbour s=%lld mu=%d", s, mu);
                CHECK(cb[q] == b[q], "backward neighbour s=%lld mu=%d", s, mu);
            }
            CHECK(((wrap >> mu) & 1u) == (unsigned)wf, "forward wrap s=%lld mu=%d", s, mu);
            CHECK(((wrap >> (4 + mu)) & 1u) == (unsigned)wb, "backward wrap s=%lld mu=%d", s, mu);
        }
    }
}

static void check_s44(const Geo& g) {
    const long long nblocks = (long long)g.nb[0] * g.nb[1] * g.nb[2] * g.nb[3];
    for (int colour = 0; colour < 2; ++colour) {
        std::set<long long> blocks;
        for (long long j = 0; j < nblocks / 2; ++j) {
            for (int l = 0; l < 256; ++l) {
                S44Site t;
                s44_setup(g, colour, j, l, t);
                int c[4];
                coords_of(g, t.s, c);
                if (l == 0) {
                    CHECK(((t.B[0] + t.B[1] + t.B[2] + t.B[3]) & 1) == colour, "block colour j=%lld", j);
                    for (int a = 0; a < 4; ++a) CHECK(t.B[a] >= 0 && t.B[a] < g.nb[a], "block range j=%lld", j);
                    CHECK(blocks.insert(t.blk).second, "block %lld twice in colour %d", t.blk, colour);
                }
                for (int a = 0; a < 4; ++a) {
                    CHECK(c[a] == t.B[a] * 4 + t.L[a], "site coords j=%lld l=%d", j, l);
                }
                CHECK(t.parity == ((c[0] + c[1] + c[2] + c[3]) & 1), "parity j=%lld l=%d", j, l);
                for (int mu = 0; mu < 4; ++mu) {
                    const int a = axis(mu);
                    CHECK(t.fin[mu] == (t.L[a] < 3), "fin");
                    CHECK(t.bin[mu] == (t.L[a] > 0), "bin");
                    int f[4] = {c[0], c[1], c[2], c[3]}, b[4] = {c[0], c[1], c[2], c[3]};
                    f[a] = (f[a] + 1) % g.d[a];
                    b[a] = (b[a] + g.d[a] - 1) % g.d[a];
                    if (t.fin[mu]) {
                        int cn[4];
                        coords_of(g, t.blk * 256 + t.fsrc[mu], cn);
                        for (int q = 0; q < 4; ++q) CHECK(cn[q] == f[q], "in-block forward j=%lld l=%d mu=%d", j, l, mu);
                    } else {
                        // the upper-halo entry: wave a stages it at lane fsrc % 64
                        CHECK(t.fsrc[mu] / 64 == a, "upper halo axis j=%lld l=%d mu=%d", j, l, mu);
                        S44Site h;
                        s44_setup(g, colour, j, 64 * a + (t.fsrc[mu] % 64), h);
                        int cn[4];
                        coords_of(g, h.up_site, cn);
                        for (int q = 0; q < 4; ++q) CHECK(cn[q] == f[q], "upper halo site j=%lld l=%d mu=%d", j, l, mu);
                        CHECK(h.up_wrap == (c[a] + 1 == g.d[a]), "upper halo wrap j=%lld l=%d mu=%d", j, l, mu);
                        CHECK(h.wmu == mu, "upper halo direction");
                    }
                    if (t.bin[mu]) {
                        CHECK(t.bcol[mu] == t.bsrc[mu], "in-block backward column source j=%lld l=%d mu=%d", j, l, mu);
                        int cn[4];
                        coords_of(g, t.blk * 256 + t.bsrc[mu], cn);
                        for (int q = 0; q < 4; ++q) CHECK(cn[q] == b[q], "in-block backward j=%lld l=%d mu=%d", j, l, mu);
                    } else {
                        CHECK(t.bsrc[mu] / 64 == a, "lower halo axis j=%lld l=%d mu=%d", j, l, mu);
                        S44Site h;
                        s44_setup(g, colour, j, 64 * a + (t.bsrc[mu] % 64), h);
                        int cn[4];
                        coords_of(g, h.dn_site, cn);
                        for (int q = 0; q < 4; ++q) CHECK(cn[q] == b[q], "lower halo site j=%lld l=%d mu=%d", j, l, mu);
                        CHECK(h.dn_wrap == (c[a] == 0), "lower halo wrap j=%lld l=%d mu=%d", j, l, mu);
                        CHECK(h.wmu == mu, "lower halo direction");
                        // the halo product's slot in the block: the column's upper-face site, which
                        // has no in-block +mu neighbour and so never writes that slot itself
                        CHECK(t.bcol[mu] == h.top, "lower halo slot j=%lld l=%d mu=%d", j, l, mu);
                        S44Site o;
                        s44_setup(g, colour, j, t.bcol[mu], o);
                        CHECK(!o.fin[mu], "lower halo slot is an upper-face site j=%lld l=%d mu=%d", j, l, mu);
                        for (int q = 0; q < 4; ++q)
                            CHECK(o.L[q] == (q == a ? 3 : t.L[q]), "lower halo slot column j=%lld l=%d mu=%d", j, l, mu);
                    }
                }
            }
        }
        CHECK((long long)blocks.size() == nblocks / 2, "colour %d covers %zu of %lld blocks", colour, blocks.size(),
              nblocks / 2);
    }
}

// xcd_swizzle is a permutation of [0, n) that keeps the workgroups of one XCD
// (j mod 8 equal) on consecutive block numbers.
static void check_swizzle() {
    for (long long n = 1; n <= 200; ++n) {
        std::vector<char> hit(n, 0);
        for (long long j = 0; j < n; ++j) {
            const long long b = xcd_swizzle(j, n);
            CHECK(b >= 0 && b < n && !hit[b], "swizzle n=%lld j=%lld", n, j);
            if (b >= 0 && b < n) hit[b] = 1;
            if (j + 8 < n) CHECK(xcd_swizzle(j + 8, n) == b + 1, "swizzle neighbours n=%lld j=%lld", n, j);
        }
    }
}

int main() {
    check_swizzle();
    // lattices (T, Z, Y, X) and tiles; the last three have several blocks per axis, unequal extents
    const int cases[][8] = {
        {8, 8, 8, 8, 4, 4, 4, 4},    {8, 8, 8, 16, 4, 4, 4, 4},   {16, 8, 16, 24, 4, 4, 4, 4},
        {24, 16, 8, 8, 4, 4, 4, 4},  {8, 6, 4, 10, 4, 2, 4, 2},   {6, 4, 8, 4, 2, 4, 4, 4},
        {4, 12, 4, 4, 2, 6, 2, 2},   {8, 8, 4, 16, 4, 4, 2, 8},
    };
    for (const auto& cs : cases) {
        const Geo g = make(cs, cs + 4);
        const int before = failures;
        check_neighbours(g);
        const bool is44 = cs[4] == 4 && cs[5] == 4 && cs[6] == 4 && cs[7] == 4;
        if (is44) check_s44(g);
        std::printf("%dx%dx%dx%d tile %dx%dx%dx%d: %s%s\n", cs[0], cs[1], cs[2], cs[3], cs[4], cs[5], cs[6], cs[7],
                    failures == before ? "ok" : "FAILED", is44 ? " (with the 4^4 kernel setup)" : "");
    }
    if (failures) {
        std::printf("%d failures\n", failures);
        return 1;
    }
    std::printf("ALL OK\n");
    return 0;
}
