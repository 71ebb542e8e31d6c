// Faraday's half step for one cell (the B update of Eq. 19 over h = dt/2):
// shared by the field advance (k_field.hip) and the push kernel, which forms
// the step's first half step for its tile from the E/B halo it has staged,
// so both give B bit for bit alike.
#pragma once

#include <hip/hip_runtime.h>

namespace pic {

struct BCell {
    float x, y, z;
};

// B - h curl E at one cell from B there and E at the cell and at its +x and
// +y neighbours (ex_y: Ex at (i, j+1), ey_x: Ey at (i+1, j), ez_x / ez_y: Ez
// at (i+1, j) / (i, j+1)); hdx = h/dx, hdy = h/dy.
__device__ __forceinline__ BCell faraday_half(float bx, float by, float bz, float ex, float ex_y, float ey,
                                              float ey_x, float ez, float ez_x, float ez_y, float hdx, float hdy)
{
    BCell b;
    b.x = bx - hdy * (ez_y - ez);
    b.y = by + hdx * (ez_x - ez);
    b.z = bz - (hdx * (ey_x - ey) - hdy * (ex_y - ex));
    return b;
}

}  // namespace pic
