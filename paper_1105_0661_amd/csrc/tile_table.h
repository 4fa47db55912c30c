// tile_table.h -- generated from tiles.json by gen_tile_table.py; do not edit.
// Sample streams per work item of the fast FP16/BF16 worker (1, 2 or 4: work
// items of 256, 128 or 64 beams), by input type (complex int8, int16),
// product (Stokes I, IQUV; voltages take the IQUV entry), K-steps of 8
// stations (4..8) and beams per block part (at most 32, 64, 128, 256 and more).
#pragma once

namespace lbf {

constexpr int kTileBeamMax[5] = {32, 64, 128, 256, 1073741824};
constexpr unsigned char kTileStreams[2][2][5][5] = {
    {
        {   // ci8, Stokes I, K-steps 4..8
            {4, 4, 2, 1, 1},
            {4, 4, 2, 1, 1},
            {4, 4, 2, 1, 1},
            {4, 4, 2, 1, 1},
            {4, 4, 2, 1, 1}},
        {   // ci8, Stokes IQUV, K-steps 4..8
            {4, 4, 2, 1, 1},
            {4, 4, 2, 1, 1},
            {4, 4, 2, 1, 1},
            {4, 4, 2, 1, 1},
            {4, 4, 2, 1, 1}}},
    {
        {   // ci16, Stokes I, K-steps 4..8
            {4, 4, 2, 1, 1},
            {4, 4, 2, 1, 1},
            {4, 2, 2, 1, 1},
            {2, 2, 2, 1, 1},
            {2, 2, 2, 1, 1}},
        {   // ci16, Stokes IQUV, K-steps 4..8
            {4, 4, 2, 1, 1},
            {4, 4, 2, 1, 1},
            {2, 2, 2, 1, 1},
            {2, 2, 2, 1, 1},
            {2, 2, 2, 1, 1}}}};

}  // namespace lbf
