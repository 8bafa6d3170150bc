// Host walk of every work item of every phase of the fused step's tile (af_tile.h)
// through the node-level arithmetic the kernels run (af_kernels.h), with the LDS tile
// as an ordinary object.  Built with address and undefined-behaviour sanitizers
// (array subscripts checked against each declared extent), it fails on the first
// read or write outside the staged window, the centre, increment or flux arrays, or a
// global plane.  Grids: ragged, tiny (smaller than the window, so that the periodic
// wrap is a modulo) and exact multiples of the tile; every tile of each grid; node
// velocities up to 1.5 cells per step, so that feet leave the window's reach and the
// foot guard must clamp them.
//
// Build (host only, under the sanitizers): tests/test_sanitize.py.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <random>
#include <vector>

#include "af_tile.h"

using namespace af;

static int g_fail = 0;

#define REQUIRE(cond, ...)                                   \
    do {                                                     \
        if (!(cond)) {                                       \
            std::fprintf(stderr, __VA_ARGS__);               \
            std::fprintf(stderr, "\n");                      \
            ++g_fail;                                        \
            return;                                          \
        }                                                    \
    } while (0)

template <class T, int TX, int TY, int RW, int NT>
static void walk_grid(int nx, int ny, double vmax, unsigned seed, int scheme) {
    using Tile = FusedTile<T, TX, TY>;
    std::unique_ptr<Tile> L(new Tile());
    std::mt19937 rng(seed);
    std::uniform_real_distribution<double> U(-1.0, 1.0);
    const PolAbs<T> pol{T(1.4), T(1.0 / 0.4)};
    const T lam1 = T(0.3), lam0 = T(0.15);
    const size_t N = (size_t)nx * ny;
    const int tiles_x = (nx + TX - 1) / TX, tiles_y = (ny + TY - 1) / TY;
    const bool onex = nx >= Tile::PX, oney = ny >= Tile::PY;
    for (int ty = 0; ty < tiles_y; ++ty)
        for (int tx = 0; tx < tiles_x; ++tx) {
            const int i0 = tx * TX, j0 = ty * TY;
            unsigned st = 0;
            // phase 0: staged primitives, with the global index the kernel forms
            for (int e = 0; e < Tile::PX * Tile::PY + NT; ++e) {
                int x, y;
                if (!Tile::stage_item(e, x, y)) continue;
                const size_t g = (size_t)wrap_win(j0 + y - 2, ny, oney) * nx + wrap_win(i0 + x - 2, nx, onex);
                REQUIRE(g < N, "stage: global index %zu outside %zu (grid %dx%d, tile %d,%d)", g, N, nx, ny, i0, j0);
                for (int k = 0; k < 12; ++k) {
                    const int var = k % 4;
                    T v = var == 0 || var == 3 ? T(1.0 + 0.1 * U(rng)) : T(vmax / (double)lam1 * U(rng));
                    L->P[k][y][x] = v;
                }
            }
            // phase 1: centres
            {
                LdsAcc<T, TX, TY> A{L.get()};
                for (int e = 0; e < Tile::SC * Tile::CY + NT; ++e) {
                    int x, y;
                    if (!Tile::centre_item(e, x, y)) continue;
                    const size_t g = (size_t)wrap_win(j0 + y, ny, oney) * nx + wrap_win(i0 + x, nx, onex);
                    REQUIRE(g < N, "centre: global index %zu outside %zu", g, N);
                    const T Ub[4] = {T(1), T(0.1), T(-0.1), T(2.6)};
                    const Prim<T> w = pol.centre(Ub, A.node(F_V, x, y), A.node(F_V, x + 1, y), A.node(F_V, x, y + 1),
                                                 A.node(F_V, x + 1, y + 1), A.node(F_EH, x, y), A.node(F_EH, x, y + 1),
                                                 A.node(F_EV, x, y), A.node(F_EV, x + 1, y));
                    (void)w;
                    // the centre of a smooth state, kept physical for the later phases
                    L->C[0][y + 2][x + 2] = T(1);
                    L->C[1][y + 2][x + 2] = T(vmax / (double)lam1 * U(rng));
                    L->C[2][y + 2][x + 2] = T(vmax / (double)lam1 * U(rng));
                    L->C[3][y + 2][x + 2] = T(1);
                }
            }
            // phase 2: increments of both durations
            {
                LdsAcc<T, TX, TY> A{L.get()};
                for (int e = 0; e < Tile::SD * Tile::DY + NT; ++e) {
                    int x, y;
                    if (!Tile::incr_item(e, x, y)) continue;
                    T d[2][3];
                    node_increments<F_V>(A, x, y, pol, lam0, lam1, d, st);
                    for (int t = 0; t < 2; ++t)
                        for (int v = 0; v < 3; ++v) L->D[t][0 * 3 + v][y + 1][x + 1] = d[t][v];
                    node_increments<F_EV>(A, x, y, pol, lam0, lam1, d, st);
                    for (int t = 0; t < 2; ++t)
                        for (int v = 0; v < 3; ++v) L->D[t][1 * 3 + v][y + 1][x + 1] = d[t][v];
                    node_increments<F_EH>(A, x, y, pol, lam0, lam1, d, st);
                    for (int t = 0; t < 2; ++t)
                        for (int v = 0; v < 3; ++v) L->D[t][2 * 3 + v][y + 1][x + 1] = d[t][v];
                    node_increments<F_C>(A, x, y, pol, lam0, lam1, d, st);
                    for (int t = 0; t < 2; ++t)
                        for (int v = 0; v < 3; ++v) L->D[t][3 * 3 + v][y + 1][x + 1] = d[t][v];
                }
            }
            // phase 3: point updates (feet gathered from the staged window and the
            // increments), then the flux store aliasing the increment buffer
            using Pts = typename Tile::template Points<RW>;
            std::vector<int> fams, xs, ys;
            {
                LdsAcc<T, TX, TY> A{L.get()};
                LdsInc<T, TX, TY> D0{L.get(), 0}, D1{L.get(), 1};
                for (int e = 0; e < Pts::N + NT; ++e) {
                    int fam, x, y;
                    if (!Pts::item(e, fam, x, y)) continue;
                    REQUIRE(x >= 0 && x <= TX && y >= 0 && y <= TY, "point item (%d, %d) outside [0, T]", x, y);
                    Prim<T> wh, w1;
                    if (scheme == 0) point_update_pair_f<0>(A, D0, D1, fam, x, y, pol, lam0, lam1, st, wh, w1);
                    else point_update_pair_f<1>(A, D0, D1, fam, x, y, pol, lam0, lam1, st, wh, w1);
                    const bool own = x < TX && y < TY && i0 + x < nx && j0 + y < ny;
                    if (own) {
                        const size_t g = (size_t)(j0 + y) * nx + (i0 + x);
                        REQUIRE(g < N, "point store: global index %zu outside %zu", g, N);
                    }
                    fams.push_back(fam);
                    xs.push_back(x);
                    ys.push_back(y);
                }
            }
            for (size_t q = 0; q < fams.size(); ++q) {
                const int x = xs[q], y = ys[q];
                if (fams[q] == F_V)
                    for (int k = 0; k < 8; ++k) L->F.FV[k][y][x] = T(0.5);
                else if (fams[q] == F_EV)
                    for (int k = 0; k < 4; ++k) L->F.FE[k][y][x] = T(0.5);
                else
                    for (int k = 0; k < 4; ++k) L->F.GE[k][y][x] = T(0.5);
            }
            // phase 4: average update of the owned cells
            for (int e = 0; e < TX * TY + NT; ++e) {
                int x, y;
                if (!Tile::update_item(e, x, y)) continue;
                if (i0 + x >= nx || j0 + y >= ny) continue;
                const size_t g = (size_t)(j0 + y) * nx + (i0 + x);
                REQUIRE(g < N, "update: global index %zu outside %zu", g, N);
                T acc = T(0);
                for (int k = 0; k < 4; ++k)
                    acc += L->F.FV[k][y][x] + L->F.FE[k][y][x] + L->F.FV[k][y + 1][x] + L->F.FV[k][y][x + 1] +
                           L->F.FE[k][y][x + 1] + L->F.FV[k][y + 1][x + 1] + L->F.FV[4 + k][y][x] +
                           L->F.GE[k][y][x] + L->F.GE[k][y + 1][x] + L->F.FV[4 + k][y + 1][x + 1];
                REQUIRE(std::isfinite((double)acc), "update: flux sum not finite");
            }
            // feet beyond one cell were clamped and flagged, never followed
            if (vmax >= 1.0) REQUIRE((st & SB_FOOT) != 0, "large velocities did not raise the foot flag");
        }
}

int main() {
    const int grids[][2] = {{4, 4}, {5, 7}, {7, 5}, {37, 29}, {70, 9}, {9, 70}, {31, 10}, {62, 20}, {33, 12}, {24, 13}};
    unsigned seed = 1;
    for (const auto& gr : grids)
        for (double vmax : {0.4, 0.95, 1.5})
            for (int scheme = 0; scheme < 2; ++scheme) {
                // the single-grid tiles (31 x 10, target rows of 32 lanes) in both precisions, and a
                // tight-row tile
                walk_grid<double, 31, 10, 32, 512>(gr[0], gr[1], vmax, seed++, scheme);
                walk_grid<float, 31, 10, 32, 512>(gr[0], gr[1], vmax, seed++, scheme);
                walk_grid<float, 24, 13, 0, 512>(gr[0], gr[1], vmax, seed++, scheme);
                // the batched kernel's candidate shapes at the extremes of their aspect ratio
                walk_grid<float, 64, 8, 0, 512>(gr[0], gr[1], vmax, seed++, scheme);
                walk_grid<float, 16, 16, 0, 256>(gr[0], gr[1], vmax, seed++, scheme);
                if (g_fail) return 1;
            }
    std::printf("tile walk: all items in bounds\n");
    return 0;
}
