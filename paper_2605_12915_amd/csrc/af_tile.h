// Layout of the fused step's LDS tile and the work items of its phases: host and
// device code, so that a host build can walk every item of every phase through the
// node-level arithmetic with bounds-checked arrays (tests/tile_bounds.cpp).
#pragma once
#include <hip/hip_runtime.h>

#include "af_kernels.h"

namespace af {

// P, C and D share one row stride (PX), and phases 1 and 2 walk their items in rows of
// that stride (the items past a region's width idle), so the lanes of a wave read
// consecutive LDS words of every plane instead of colliding on banks where the rows of
// the item grid and of the array wrap at different widths (FP64 2% faster; FP32 4.6%,
// its bank-conflict cycles had outnumbered its active LDS cycles).
template <class T, int TX, int TY>
struct FusedTile {
    static constexpr int PX = TX + 5, PY = TY + 5;   // primitives: cells [-2, T+3)
    static constexpr int CX = TX + 4, CY = TY + 4;   // centres:    cells [-2, T+2)
    static constexpr int DX = TX + 3, DY = TY + 3;   // increments: node-cells [-1, T+2)
    static constexpr int VX = TX + 1, VY = TY + 1;   // flux nodes: node-cells [0, T]
    static constexpr int SC = PX, SD = PX;           // row strides of C, D
    T P[12][PY][PX];
    T C[4][CY][SC];
    union {
        T D[2][12][DY][SD];                          // [tau][fam*3 + var]
        struct {
            T FV[8][VY][VX];                         // V nodes: F~ (0..3), G~ (4..7)
            T FE[4][TY][VX];                         // Ev nodes: F~
            T GE[4][VY][TX];                         // Eh nodes: G~
        } F;
    };

    // Work items of the phases (item e of a workgroup's round-robin walk):
    // phase 0 stages node-cell (x, y) of P (cells x - 2, y - 2 of the tile),
    static AF_HD bool stage_item(int e, int& x, int& y) {
        x = e % PX;
        y = e / PX;
        return e < PX * PY;
    }
    // phase 1 recovers the centre of tile cell (x, y), x, y in [-2, T + 2),
    static AF_HD bool centre_item(int e, int& x, int& y) {
        x = e % SC - 2;
        y = e / SC - 2;
        return e < SC * CY && x + 2 < CX;
    }
    // phase 2 the increments of node-cell (x, y), x, y in [-1, T + 2),
    static AF_HD bool incr_item(int e, int& x, int& y) {
        x = e % SD - 1;
        y = e / SD - 1;
        return e < SD * DY && x + 1 < DX;
    }
    // phase 3 the point update of target family fam at node-cell (x, y) in [0, T]: V
    // targets (VX x VY), then Ev (VX x TY), then Eh (TX x VY), each family in rows of
    // RW lanes (0: rows as wide as the family's row of targets; lanes past it idle),
    template <int RW>
    struct Points {
        static constexpr int WV = RW ? RW : VX, WE = RW ? RW : VX, WH = RW ? RW : TX;
        static constexpr int NV = WV * VY, NE = WE * TY, NH = WH * VY, N = NV + NE + NH;
        static AF_HD bool item(int e, int& fam, int& x, int& y) {
            if (e >= N) return false;
            if (e < NV) { fam = F_V; x = e % WV; y = e / WV; return x < VX; }
            if (e < NV + NE) { fam = F_EV; x = (e - NV) % WE; y = (e - NV) / WE; return x < VX; }
            fam = F_EH; x = (e - NV - NE) % WH; y = (e - NV - NE) / WH;
            return x < TX;
        }
    };
    // and phase 4 updates the average of tile cell (x, y).
    static AF_HD bool update_item(int e, int& x, int& y) {
        x = e % TX;
        y = e / TX;
        return e < TX * TY;
    }
};

template <class T, int TX, int TY>
struct LdsAcc {
    const FusedTile<T, TX, TY>* t;
    AF_HD Prim<T> node(int fam, int x, int y) const {
        if (fam == F_C) return {t->C[0][y + 2][x + 2], t->C[1][y + 2][x + 2], t->C[2][y + 2][x + 2], t->C[3][y + 2][x + 2]};
        const int b = 4 * fam;
        return {t->P[b][y + 2][x + 2], t->P[b + 1][y + 2][x + 2], t->P[b + 2][y + 2][x + 2], t->P[b + 3][y + 2][x + 2]};
    }
};

template <class T, int TX, int TY>
struct LdsInc {
    const FusedTile<T, TX, TY>* t;
    int tau;
    AF_HD T inc(int fam, int x, int y, int var) const {
        return t->D[tau][fam * 3 + var][y + 1][x + 1];
    }
};

AF_HD int wrap_any(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

// Periodic index of the tile window: one conditional shift when the grid is at least
// as large as the window (the usual case, decided per launch), else a modulo.
AF_HD int wrap_win(int v, int n, bool one) {
    if (one) return v < 0 ? v + n : (v >= n ? v - n : v);
    return wrap_any(v, n);
}

}  // namespace af
