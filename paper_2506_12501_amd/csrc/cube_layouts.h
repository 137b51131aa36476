// cube_layouts.h -- written by gen_cube_layouts.py; do not edit.
// Compact [r]^(0) table layouts: entry (t, u, v), t + u + v <= D - 1, at
// t*ST + u*SU + v; tables of successive quartets SIZE doubles apart; valid
// (every entry of up to 48 tables at its own address) for D = 1..25.
#pragma once

namespace mdx {

constexpr int CUBE_COMPACT_QMAX = 48;
constexpr int CUBE_COMPACT_DMAX = 25;
// {D, SU, ST, SIZE}
constexpr int CUBE_COMPACT[25][4] = {
    {1, 1, 1, 1},
    {2, 2, 3, 4},
    {3, 4, 6, 13},
    {4, 5, 12, 32},
    {5, 9, 29, 62},
    {6, 11, 28, 114},
    {7, 11, 72, 159},
    {8, 10, 72, 262},
    {9, 20, 112, 363},
    {10, 10, 93, 512},
    {11, 11, 120, 659},
    {12, 26, 171, 889},
    {13, 13, 164, 1063},
    {14, 18, 203, 1356},
    {15, 30, 218, 1758},
    {16, 20, 265, 2028},
    {17, 18, 299, 2537},
    {18, 19, 340, 2898},
    {19, 22, 409, 3493},
    {20, 22, 377, 3980},
    {21, 22, 441, 4641},
    {22, 24, 515, 5436},
    {23, 48, 553, 6143},
    {24, 26, 607, 7010},
    {25, 52, 651, 7877},
};

}  // namespace mdx
