// geometry.cpp -- per-ray sweep tables (host, double precision -> fixed point).
#include "geometry.h"

#include <algorithm>
#include <cmath>

namespace eptv {

RayFx HostRay::fx() const
{
    RayFx r;
    r.step = S;
    r.span = S < 0 ? -S : S;
    r.lo0 = S < 0 ? E0 + S : E0;
    r.w32 = w32;
    r.wfull = rows ? -wfull : wfull;
    return r;
}

// ------------------------------------------------------------------ geometry
// Ray (v, b) leaves the source s_v = -SAD (cos theta_v, sin theta_v) along
// theta_v + beta_b (Sec. 3 scanner; App. III Eq. A6).  Its sweep form is
// computed in double precision and stored in 32.32 fixed point (see RayTable).
static long long to_fixed(double e) { return std::llround(std::ldexp(e, 32)); }

HostRay make_ray(const Plan& p, double theta, double beta)
{
    const double d = p.pixel;
    const double c = std::cos(theta + beta), s = std::sin(theta + beta);
    const double sx = -p.sad * std::cos(theta), sy = -p.sad * std::sin(theta);
    const double x0 = -0.5 * p.nx * d, y0 = -0.5 * p.ny * d;
    HostRay R;
    double e0, slope;
    int ncross, nsweep;
    if (std::fabs(c) >= std::fabs(s)) {  // swept column by column
        e0 = (sy + (x0 - sx) * s / c - y0) / d;
        slope = s / c;
        R.w32 = s != 0.0 ? (float)std::ldexp(d / std::fabs(s), -32) : 0.0f;
        R.wfull = (float)(d / std::fabs(c));
        R.rows = false;
        ncross = p.ny;
        nsweep = p.nx;
    } else {  // swept row by row
        e0 = (sx + (y0 - sy) * c / s - x0) / d;
        slope = c / s;
        R.w32 = c != 0.0 ? (float)std::ldexp(d / std::fabs(c), -32) : 0.0f;
        R.wfull = (float)(d / std::fabs(s));
        R.rows = true;
        ncross = p.nx;
        nsweep = p.ny;
    }
    R.E0 = to_fixed(e0);
    R.S = to_fixed(slope);
    // Sweep cells whose entry/exit coordinates can touch [0, ncross), widened
    // far beyond the fixed-point rounding of e.
    const double delta = std::ldexp(1.0, -18) * (p.nx + p.ny + 2);
    if (R.S == 0) {
        const double e = std::ldexp((double)R.E0, -32);
        const bool in = e >= -delta && e < ncross + delta;
        R.k_lo = 0;
        R.k_hi = in ? nsweep : 0;
    } else {
        double ka = (-delta - e0) / slope, kb = (ncross + delta - e0) / slope;
        double lo = std::floor(std::min(ka, kb)) - 1.0, hi = std::ceil(std::max(ka, kb)) + 1.0;
        lo = std::min(std::max(lo, 0.0), (double)nsweep);
        hi = std::min(std::max(hi, 0.0), (double)nsweep);
        R.k_lo = (int)lo;
        R.k_hi = std::max((int)hi, R.k_lo);
    }
    return R;
}

}  // namespace eptv
