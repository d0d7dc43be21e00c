// Pieces of the host operator builder (builder.cpp) that the TT-format
// construction of the same operators (ttbuild.hip) reuses.
#pragma once
#include "host_linalg.h"

// MPO (d = 4) of the 2D shift u(i + di, j + dj) on the 2^n x 2^n grid, zero outside
// 0 <= i + di < 2^n, periodic in j, in bit order `order` (QTT_ORDER_*): a carry
// automaton of bond 4 (Sec. 2.1.2).
HostTT cyl_shift_mpo(int n, int di, int dj, int order);

// Radius of grid row i (i = -2 .. 2^n + 1) of the O-grid around the unit cylinder
// (App. E): row -1 is the wall (r = 0.5), row 2^n the far field (r = r_out).
double cyl_row_radius(int i, int n, double r_out);
