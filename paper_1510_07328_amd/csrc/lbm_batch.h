// Internal descriptors of the batched tube sweep (device-visible, plain data).
#pragma once

#include <cstdint>

namespace lbm {

struct BatchTube {
    int64_t off;     // element offset of the tube's populations in a buffer (9 x 4 x nx values)
    int nx;          // columns
    int steps;       // steps of the current schedule
    int cur;         // buffer (0 / 1) holding the tube's state
    int pad;
    double omega;    // 1 / tau
    double n_left, n_right;
};

struct BatchTile {
    int tube;  // index into the tube table
    int x0;    // first column of the tile
    int s;     // columns in the tile
    int pad;
};

}  // namespace lbm
