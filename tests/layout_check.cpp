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
            // even-odd halves: the parity-p member of pair h has half index h
            if (wd::eo_supported(g))
                for (int h = 0; h < g.V / 2; ++h)
                    for (int p = 0; p < 2; ++p) {
                        const int i = wd::site_of_half(g, h, p);
                        int x, y, z, t;
                        wd::coords_of(g, i, x, y, z, t);
                        if ((i >> 1) != h || ((x + y + z + t) & 1) != p) ++fails;
                    }
            // the marching half-field stencil's entries: each output entry of
            // either parity once, its t neighbours where the images hold
            // them, and the partials within the capacity
            if (wd::eo_supported(g))
                for (int prec = 0; prec < 3; ++prec) {
                    const int w = wd::eo_wvol(g, prec);
                    if (!w) continue;
                    const int hvol = g.bvol / 2, nsub = hvol / w;
                    const int ncols = g.V / (Lt * g.bvol);
                    if (hvol % w || w % 64 || w > wd::kTmMaxBlock) ++fails;
                    if ((long long)(g.V / 2 / w) > wd::reduce_partials_cap(g, 1)) ++fails;
                    for (int ch : {1, 3, Lt}) {
                        const int nch = (Lt + ch - 1) / ch;
                        for (int p = 0; p < 2; ++p) {
                            std::vector<int> out(g.V / 2, 0);
                            for (int cb = 0; cb < ncols * nch * nsub; ++cb) {
                                const int cc = cb / nsub, hp = cb % nsub;
                                const int chunk = cc / ncols, col = cc % ncols;
                                const int t0 = chunk * ch, t1 = t0 + ch < Lt ? t0 + ch : Lt;
                                const int hbase = col * Lt * hvol + hp * w;
                                if (hbase % 64) ++fails;
                                for (int l = 0; l < w; ++l) {
                                    const int tp = t0 == 0 ? Lt - 1 : t0 - 1;
                                    const int i0 = wd::site_of_half(g, hbase + t0 * hvol + l, p);
                                    if ((wd::neighbours(g, i0).tm >> 1) != hbase + tp * hvol + l) ++fails;
                                    for (int t = t0; t < t1; ++t) {
                                        const int H = hbase + t * hvol + l;
                                        if (H < 0 || H >= g.V / 2) { ++fails; continue; }
                                        out[H]++;
                                        const int i = wd::site_of_half(g, H, p);
                                        const wd::Nbrs n = wd::neighbours(g, i);
                                        const int tn = t + 1 < Lt ? t + 1 : 0;
                                        if ((n.tp >> 1) != hbase + tn * hvol + l) ++fails;
                                        if (wd::site_of_half(g, n.tp >> 1, 1 - p) != n.tp) ++fails;
                                        if (t + 1 < t1) {
                                            const int i1 = wd::site_of_half(g, H + hvol, p);
                                            if ((wd::neighbours(g, i1).tm >> 1) != H) ++fails;
                                        }
                                    }
                                }
                            }
                            for (int h = 0; h < g.V / 2; ++h)
                                if (out[h] != 1) ++fails;
                        }
                    }
                }
            // reduction partials: room for every reducing launch shape (a
            // launch writes index block * nrhs + rhs for each of its blocks
            // per rhs)
            for (int nrhs = 1; nrhs <= 12; ++nrhs) {
                const long long cap = wd::reduce_partials_cap(g, nrhs);
                if ((long long)wd::site_blocks(g.V) * nrhs > cap) ++fails;
                if (wd::tm_eligible(g)) {
                    for (int prec = 0; prec < 3; ++prec) {
                        const int w = wd::tm_wvol(g, prec);
                        if (w % 64 || g.bvol % w || w > wd::kTmMaxBlock) ++fails;
                        if ((long long)(g.V / w) * nrhs > cap) ++fails;
                    }
                    // chunks tile the time extent
                    for (int env = 0; env <= Lt + 1; ++env) {
                        const int ch = wd::tm_chunk_len(g, nrhs, env);
                        if (ch < 1 || ch > Lt) ++fails;
                        if ((long long)wd::tm_blocks(g, ch) * ch < (long long)(g.V / g.bvol)) ++fails;
                    }
                }
                // the last entry of the last rhs lies inside the field
                for (int prec = 0; prec < 3; ++prec) {
                    const size_t tb = wd::spinor_tile_bytes(prec);
                    const size_t rhs_bytes = (size_t)(wd::rhs_stride(g.V) / 64) * tb;
                    const size_t last = (size_t)(nrhs - 1) * rhs_bytes + (size_t)((g.V - 1) / 64) * tb + tb;
                    if (last > wd::field_data_bytes(prec, g.V, nrhs)) ++fails;
                    if (wd::rhs_stride(g.V) % 64 || wd::rhs_stride(g.V) < g.V) ++fails;
                }
            }
        }
      }
    }
    if (fails) printf("lattice %dx%dx%dx%d: %d mismatches\n", Lx, Ly, Lz, Lt, fails);
    return fails;
}

// the default brick choice divides the lattice and gives whole tiles
static int check_choice(int Lx, int Ly, int Lz, int Lt) {
    wd::Geom g{};
    g.L[0] = Lx; g.L[1] = Ly; g.L[2] = Lz; g.L[3] = Lt;
    g.V = Lx * Ly * Lz * Lt;
    wd::choose_bricks(g);
    int fails = 0;
    if (Lx % g.tx || Ly % g.ty || Lz % g.tz || g.bvol != g.tx * g.ty * g.tz) ++fails;
    if (g.ncx * g.tx != Lx || g.ncy * g.ty != Ly || g.ncz * g.tz != Lz) ++fails;
    printf("bricks %dx%dx%dx%d: %dx%dx%d\n", Lx, Ly, Lz, Lt, g.tx, g.ty, g.tz);
    return fails;
}

// neighbours read from outside a site's part, against the closed forms for
// parts of whole x rows: per split direction, 2 / extent of the part in it
// (brick faces and part boundaries alike), none in a direction the brick
// spans whole
static int check_part_faces() {
    const int L[4] = {48, 48, 48, 96};
    int fails = 0;
    struct Case { int a, b, c, w, want; };
    const Case cs[] = {
        {48, 2, 4, 384, 240 * 3 / 2},  // y 1 + z 1/2
        {48, 2, 8, 192, 240 * 2},      // parts 48x2x2: y 1 + z 1
        {48, 4, 4, 192, 240 * 5 / 2},  // parts 48x4x1: y 1/2 + z 2
        {48, 1, 16, 192, 240 * 5 / 2}, // parts 48x1x4: y 2 + z 1/2
        {48, 2, 8, 768, 240 * 5 / 4},  // whole brick: y 1 + z 1/4
        {16, 4, 4, 256, 240 * 9 / 8},  // x split too: x 1/8 + y 1/2 + z 1/2
    };
    for (const Case &k : cs) {
        const int got = wd::part_faces(L, k.a, k.b, k.c, k.w);
        if (got != k.want) {
            printf("part_faces %dx%dx%d w=%d: %d, want %d\n", k.a, k.b, k.c, k.w, got, k.want);
            ++fails;
        }
    }
    // the float64 part size rule: 192 where it divides, else up to 384
    const int parts[][2] = {{768, 192}, {384, 192}, {192, 192}, {256, 256}, {320, 320},
                            {512, 256}, {64, 64}, {1024, 256}};
    for (const auto &q : parts)
        if (wd::part_sites(q[0], WD_F64) != q[1]) {
            printf("part_sites(%d) = %d, want %d\n", q[0], wd::part_sites(q[0], WD_F64), q[1]);
            ++fails;
        }
    // the GPU tests' ragged case: 4x20x20x20 with 12 rhs marches chunks of
    // 3 time slices, so the last chunk of a column has 2
    {
        wd::Geom g{};
        g.L[0] = 4; g.L[1] = 20; g.L[2] = 20; g.L[3] = 20;
        g.V = 4 * 20 * 20 * 20;
        wd::choose_bricks(g);
        for (int prec = 0; prec < 3; ++prec)
            if (!wd::tm_eligible(g) ||
                wd::tm_chunk_len(g, 12 * (g.bvol / wd::tm_wvol(g, prec)), 0) != 3) {
                printf("4x20x20x20: chunk %d, want 3\n",
                       wd::tm_chunk_len(g, 12 * (g.bvol / wd::tm_wvol(g, prec)), 0));
                ++fails;
            }
    }
    // and the even-odd one: 8x20x20x20 with 12 rhs, marching halves (float64
    // and float32) in chunks of 3
    {
        wd::Geom g{};
        g.L[0] = 8; g.L[1] = 20; g.L[2] = 20; g.L[3] = 20;
        g.V = 8 * 20 * 20 * 20;
        wd::choose_bricks(g);
        for (int prec = 0; prec < 2; ++prec) {
            const int w = wd::eo_wvol(g, prec);
            if (!w || wd::tm_chunk_len(g, 12 * (g.bvol / 2 / w), 0) != 3) {
                printf("8x20x20x20 even-odd: w %d, want a chunk of 3\n", w);
                ++fails;
            }
        }
    }
    return fails;
}

int main() {
    int f = 0;
    f += check_part_faces();
    f += check_choice(48, 48, 48, 96);
    f += check_choice(24, 24, 24, 48);
    f += check_choice(16, 16, 16, 32);
    f += check_choice(12, 12, 12, 12);
    f += check_choice(8, 8, 8, 8);
    f += check_choice(4, 4, 4, 4);
    f += check_choice(2, 4, 2, 6);
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
    f += check(16, 8, 8, 4);
    f += check(8, 8, 12, 6);
    printf(f ? "FAIL\n" : "OK\n");
    return f ? 1 : 0;
}
