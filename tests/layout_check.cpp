// Host check of the internal site order and the stencil's neighbour
// arithmetic (wd_internal.hpp) against brute force on the lattice
// coordinates, for many lattice shapes and brick extents.  Exit code 0 on
// success.
#include <cstdio>
#include <vector>

#include "runtime.hpp"

static int check(int Lx, int Ly, int Lz, int Lt) {
    int fails = 0;
    for (int tx = 1; tx <= Lx; ++tx) {
      if (Lx % tx) continue;
      for (int ty = 1; ty <= Ly; ++ty) {
        if (Ly % ty) continue;
        for (int tz = 1; tz <= Lz; ++tz) {
            if (Lz % tz) continue;
            wd::Geom g{};
            g.L[0] = Lx; g.L[1] = Ly; g.L[2] = Lz; g.L[3] = Lt;
            g.V = Lx * Ly * Lz * Lt;
            g.tx = tx; g.ty = ty; g.tz = tz;
            g.ncx = Lx / tx; g.ncy = Ly / ty; g.ncz = Lz / tz; g.bvol = tx * ty * tz;
            std::vector<int> seen(g.V, 0);
            for (int i = 0; i < g.V; ++i) {
                int x, y, z, t;
                wd::coords_of(g, i, x, y, z, t);
                if (x < 0 || x >= Lx || y < 0 || y >= Ly || z < 0 || z >= Lz || t < 0 || t >= Lt ||
                    wd::index_of(g, x, y, z, t) != i) { ++fails; continue; }
                seen[wd::lex_of(g, x, y, z, t)]++;
                wd::Nbrs n = wd::neighbours(g, i);
                const int want[8] = {
                    wd::index_of(g, (x + 1) % Lx, y, z, t), wd::index_of(g, (x + Lx - 1) % Lx, y, z, t),
                    wd::index_of(g, x, (y + 1) % Ly, z, t), wd::index_of(g, x, (y + Ly - 1) % Ly, z, t),
                    wd::index_of(g, x, y, (z + 1) % Lz, t), wd::index_of(g, x, y, (z + Lz - 1) % Lz, t),
                    wd::index_of(g, x, y, z, (t + 1) % Lt), wd::index_of(g, x, y, z, (t + Lt - 1) % Lt)};
                const int got[8] = {n.xp, n.xm, n.yp, n.ym, n.zp, n.zm, n.tp, n.tm};
                for (int k = 0; k < 8; ++k)
                    if (got[k] != want[k]) ++fails;
                if (n.cross_tp != (t == Lt - 1) || n.cross_tm != (t == 0)) ++fails;
            }
            for (int s = 0; s < g.V; ++s)
                if (seen[s] != 1) ++fails;
            // reduction partials: room for every reducing launch shape
            for (int nrhs = 1; nrhs <= 12; ++nrhs) {
                const long long cap = wd::reduce_partials_cap(g, nrhs);
                const int bs = wd::block_for_nrhs(nrhs);
                if ((long long)wd::blocks_for((long long)g.V * nrhs, bs) * nrhs > cap) ++fails;
                if (wd::tm_eligible(g, nrhs))
                    for (int ch = 1; ch <= Lt; ++ch)
                        if (wd::tm_blocks(g, ch) > cap) ++fails;
            }
        }
      }
    }
    if (fails) printf("lattice %dx%dx%dx%d: %d mismatches\n", Lx, Ly, Lz, Lt, fails);
    return fails;
}

int main() {
    int f = 0;
    f += check(2, 2, 2, 2);
    f += check(4, 4, 4, 4);
    f += check(4, 6, 8, 10);
    f += check(2, 4, 6, 8);
    f += check(8, 12, 4, 6);
    f += check(6, 4, 12, 2);
    f += check(48, 12, 4, 2);
    f += check(24, 6, 8, 4);
    f += check(12, 12, 12, 12);
    f += check(16, 16, 16, 8);
    printf(f ? "FAIL\n" : "OK\n");
    return f ? 1 : 0;
}
