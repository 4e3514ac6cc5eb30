// geometry.h -- host construction of the per-ray sweep tables and of the
// float32 system matrix they define (shared by plan creation and the stored
// matrix).
#pragma once

#include "eptv_internal.h"

namespace eptv {

struct HostRay {
    long long E0, S;  // fixed-point entry coordinate at sweep cell 0 and slope
    float w32, wfull;
    bool rows;        // swept row by row
    int k_lo, k_hi;   // sweep cells that can meet the image
    RayFx fx() const;
};

// Ray leaving the source at view angle theta along theta + beta.
HostRay make_ray(const Plan& p, double theta, double beta);

// Visit every (pixel, length) entry of the ray with a positive length, in
// sweep order, with the same arithmetic as the kernels (cell_weights).
template <class F>
void for_each_entry(const HostRay& H, const Plan& p, F&& f)
{
    const RayFx R = H.fx();
    const int ncross = H.rows ? p.nx : p.ny;
    const float wfull = H.wfull;
    for (int k = H.k_lo; k < H.k_hi; ++k) {
        const CellW w = cell_weights(R.lo0 + (long long)k * R.step, R.span, R.w32, wfull);
        for (int e = 0; e < 2; ++e) {
            const int m = w.m0 + e;
            const float c = e == 0 ? w.c0 : w.c1;
            if (m < 0 || m >= ncross || !(c > 0.0f)) continue;
            const long long pix = H.rows ? (long long)k * p.nx + m : (long long)m * p.nx + k;
            f(pix, c);
        }
    }
}

}  // namespace eptv
