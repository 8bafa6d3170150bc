// Host build of the foot-centred exact point update (af_footcentred.h, the code the
// GPU kernel runs), for the CPU comparison with the oracle (tests/test_fc_host.py).
// Reads   int32 nx, ny; double h, gamma, dt; 16 nx ny doubles (the state planes)
// writes  int32 status bits; 24 nx ny doubles: new point values after dt/2, then dt
//         (planes fam * 4 + (rho, u, v, p) per duration).
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "af_footcentred.h"

using namespace af;

struct HostAcc {
    const double* s;   // 16 planes
    const double* C;   // 4 planes of recovered centres (may be null while computing them)
    int nx, ny;
    size_t idx(int i, int j) const {
        i = ((i % nx) + nx) % nx;
        j = ((j % ny) + ny) % ny;
        return (size_t)j * nx + i;
    }
    Prim<double> node(int fam, int i, int j) const {
        const size_t k = idx(i, j), N = (size_t)nx * ny;
        if (fam == F_C) return {C[k], C[N + k], C[2 * N + k], C[3 * N + k]};
        const int b = 4 + 4 * fam;
        return {s[b * N + k], s[(b + 1) * N + k], s[(b + 2) * N + k], s[(b + 3) * N + k]};
    }
};

int main(int argc, char** argv) {
    if (argc != 3) { std::fprintf(stderr, "usage: fc_host in out\n"); return 2; }
    FILE* f = std::fopen(argv[1], "rb");
    if (!f) return 2;
    int nx = 0, ny = 0;
    double h = 0, gamma = 0, dt = 0;
    if (std::fread(&nx, 4, 1, f) != 1 || std::fread(&ny, 4, 1, f) != 1 || std::fread(&h, 8, 1, f) != 1 ||
        std::fread(&gamma, 8, 1, f) != 1 || std::fread(&dt, 8, 1, f) != 1)
        return 2;
    const size_t N = (size_t)nx * ny;
    std::vector<double> s(16 * N), C(4 * N), out(24 * N);
    if (std::fread(s.data(), 8, s.size(), f) != s.size()) return 2;
    std::fclose(f);
    HostAcc A{s.data(), C.data(), nx, ny};
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const size_t c = (size_t)j * nx + i;
            const double Ub[4] = {s[c], s[N + c], s[2 * N + c], s[3 * N + c]};
            const Prim<double> w = recover_centre(Ub, A.node(F_V, i, j), A.node(F_V, i + 1, j), A.node(F_V, i, j + 1),
                                                  A.node(F_V, i + 1, j + 1), A.node(F_EH, i, j), A.node(F_EH, i, j + 1),
                                                  A.node(F_EV, i, j), A.node(F_EV, i + 1, j), gamma);
            C[c] = w.r; C[N + c] = w.u; C[2 * N + c] = w.v; C[3 * N + c] = w.p;
        }
    unsigned st = 0;
    for (int t = 0; t < 2; ++t) {
        const double lam = (t == 0 ? 0.5 * dt : dt) / h;
        for (int fam = 0; fam < 3; ++fam)
            for (int j = 0; j < ny; ++j)
                for (int i = 0; i < nx; ++i) {
                    const Prim<double> w = fc_point_update(A, fam, i, j, gamma, lam, st);
                    const size_t c = (size_t)j * nx + i, b = (size_t)(12 * t + 4 * fam) * N;
                    out[b + c] = w.r; out[b + N + c] = w.u; out[b + 2 * N + c] = w.v; out[b + 3 * N + c] = w.p;
                }
    }
    FILE* g = std::fopen(argv[2], "wb");
    if (!g) return 2;
    const int sti = (int)st;
    std::fwrite(&sti, 4, 1, g);
    std::fwrite(out.data(), 8, out.size(), g);
    std::fclose(g);
    return 0;
}
