// tables.cpp -- host-only construction of a plan's tables (see tables.h).
#include "tables.h"

#include <algorithm>
#include <cmath>
#include <cstring>

#include "geometry.h"

namespace eptv {

Plan host_plan(const eptv_geometry* g)
{
    Plan p;
    p.nx = g->nx;
    p.ny = g->ny;
    p.V = g->n_views;
    p.B = g->n_bins;
    p.pixel = g->pixel_mm;
    p.dbeta = g->dbeta_rad;
    p.bin_offset = g->bin_offset;
    p.sad = g->sad_mm;
    p.sdd = g->sdd_mm;
    p.angles.resize(p.V);
    for (int v = 0; v < p.V; ++v) p.angles[v] = g->view_angles_rad ? g->view_angles_rad[v] : 2.0 * M_PI * v / p.V;
    return p;
}

int validate_geometry(const eptv_geometry* g)
{
    if (!g) return EPTV_ERR_ARG;
    // at least 2 x 2 pixels: the projector reads a cell's two pixels as one pair
    if (g->nx < 2 || g->ny < 2 || g->n_views <= 0 || g->n_bins <= 0) return EPTV_ERR_ARG;
    if (g->nx > 32768 || g->ny > 32768 || (long long)g->n_views * g->n_bins > (1LL << 30)) return EPTV_ERR_ARG;
    if (!(g->pixel_mm > 0) || !std::isfinite(g->pixel_mm)) return EPTV_ERR_GEOMETRY;
    if (!(g->dbeta_rad > 0) || !std::isfinite(g->dbeta_rad) || !std::isfinite(g->bin_offset))
        return EPTV_ERR_GEOMETRY;
    const double half_diag = 0.5 * g->pixel_mm * std::sqrt((double)g->nx * g->nx + (double)g->ny * g->ny);
    if (!(g->sad_mm > half_diag * (1.0 + 1e-6)) || !std::isfinite(g->sad_mm)) return EPTV_ERR_GEOMETRY;
    if (!(g->sdd_mm >= g->sad_mm)) return EPTV_ERR_GEOMETRY;
    const double edge = (0.5 * (g->n_bins - 1) + std::fabs(g->bin_offset)) * g->dbeta_rad;
    // every ray, and the angle one bin beyond each detector end, points into the half-plane ahead
    if (!(edge + g->dbeta_rad < 0.5 * M_PI)) return EPTV_ERR_GEOMETRY;
    if (g->view_angles_rad)
        for (int v = 0; v < g->n_views; ++v)
            if (!std::isfinite(g->view_angles_rad[v])) return EPTV_ERR_GEOMETRY;
    return EPTV_OK;
}

// eps of Eq. A3 as the P2 kernels use it: its float square must be a positive
// normal number, so every half-edge magnitude is at least eps > 0 and the
// fluxes of Eq. A2 (which divide by the magnitude) stay finite on flat regions.
bool tv_eps_ok(double eps)
{
    const float e2 = (float)(eps * eps);
    return eps > 0 && std::isnormal(e2);
}

int check_params(const eptv_params* q)
{
    if (!q) return EPTV_ERR_ARG;
    if (q->tv_iters > 0 && !tv_eps_ok(q->tv_eps)) return EPTV_ERR_ARG;
    if (q->outer_iters < 0 || q->cgls_iters < 0 || q->cgls_iters > kMaxCgls || q->tv_iters < 0) return EPTV_ERR_ARG;
    if (q->tv_iters > 0 && !(q->lambda > 0)) return EPTV_ERR_ARG;
    if (q->cgls_iters == 0 && !(q->mu >= 0 && q->lambda > 0)) return EPTV_ERR_ARG;
    if (q->sigma_fixed < 0 && !(q->edge_quantile > 0 && q->edge_quantile <= 1)) return EPTV_ERR_ARG;
    if (std::isnan(q->sigma_fixed) || !(q->tv_eps >= 0) || !(q->sigma_floor > 0)) return EPTV_ERR_ARG;
    if (q->tv_iters > 0 && (!(q->armijo_shrink > 0 && q->armijo_shrink < 1) || q->armijo_max_backtracks < 0 ||
                            q->armijo_max_backtracks > 4096 || !(q->armijo_c >= 0)))
        return EPTV_ERR_ARG;
    if ((long long)q->outer_iters * q->tv_iters > (1LL << 28)) return EPTV_ERR_ARG;
    if ((long long)q->outer_iters * q->cgls_iters > (1LL << 28)) return EPTV_ERR_ARG;
    if (q->check_finite != 0 && q->check_finite != 1) return EPTV_ERR_ARG;
    if (q->stored_matrix < 0 || q->stored_matrix > 2 || (q->interp_bp != 0 && q->interp_bp != 1))
        return EPTV_ERR_ARG;
    if (q->check_every < 0 || !(q->stop_rmse >= 0) || !std::isfinite(q->stop_rmse)) return EPTV_ERR_ARG;
    return EPTV_OK;
}

uint32_t select_rank(const Plan& p, double q)
{
    const double n = (double)n_edges(p);
    long long k = (long long)std::ceil(q * n) - 1;
    k = std::max(0LL, std::min(k, (long long)n - 1));
    return (uint32_t)k;
}

float t0_of(const eptv_params& q)
{
    return (float)(q.armijo_t0 > 0 ? q.armijo_t0 : 1.0 / q.lambda);
}

// sigma the per-iteration state starts from: fixed, or -1 (chosen by the selection)
float sigma_init(const eptv_params& q) { return q.sigma_fixed < 0 ? -1.0f : (float)q.sigma_fixed; }

size_t n_edges(const Plan& p) { return (size_t)p.ny * (p.nx + 1) + (size_t)(p.ny + 1) * p.nx; }

// Per tile, every ray that can meet one of its pixels, as global ray ids
// (views ascending, bins ascending within a view).  The pixel centres span a
// rectangle, so their angles seen from the source lie between those of its
// corners; a ray through a pixel passes within d/sqrt(2) of its centre, i.e.
// within asin(rad / l) of the centre's angle, largest at the rectangle point
// nearest the source; half a bin more covers rounding.
void bp_tile_lists(const Plan& p, std::vector<int>& off, std::vector<int>& list)
{
    const int gx = (p.nx + kBpTile - 1) / kBpTile, gy = (p.ny + kBpTile - 1) / kBpTile;
    const double rad = p.pixel * std::sqrt(0.5) * (1.0 + 1e-6), bin_c = 0.5 * (p.B - 1) - p.bin_offset;
    off.assign((size_t)gx * gy + 1, 0);
    list.clear();
    for (int ty = 0; ty < gy; ++ty)
        for (int tx = 0; tx < gx; ++tx) {
            const int i0 = tx * kBpTile, i1 = std::min(i0 + kBpTile, p.nx) - 1;
            const int j0 = ty * kBpTile, j1 = std::min(j0 + kBpTile, p.ny) - 1;
            const double x0 = (i0 + 0.5 - 0.5 * p.nx) * p.pixel, x1 = (i1 + 0.5 - 0.5 * p.nx) * p.pixel;
            const double y0 = (j0 + 0.5 - 0.5 * p.ny) * p.pixel, y1 = (j1 + 0.5 - 0.5 * p.ny) * p.pixel;
            for (int v = 0; v < p.V; ++v) {
                const double cs = std::cos(p.angles[v]), sn = std::sin(p.angles[v]);
                const double sx = -p.sad * cs, sy = -p.sad * sn;
                double lo = 1e300, hi = -1e300;
                for (int cnr = 0; cnr < 4; ++cnr) {
                    const double px = (cnr & 1) ? x1 : x0, py = (cnr & 2) ? y1 : y0;
                    const double along = px * cs + py * sn + p.sad, across = py * cs - px * sn;
                    const double b = std::atan2(across, along) / p.dbeta + bin_c;
                    lo = std::min(lo, b);
                    hi = std::max(hi, b);
                }
                const double nxp = std::min(std::max(sx, x0), x1) - sx, nyp = std::min(std::max(sy, y0), y1) - sy;
                const double lmin = std::sqrt(nxp * nxp + nyp * nyp);
                const double hw = std::asin(std::min(1.0, rad / lmin)) / p.dbeta + 0.5;
                const long long b0 = std::max(0LL, (long long)std::floor(lo - hw));
                const long long b1 = std::min((long long)p.B - 1, (long long)std::ceil(hi + hw));
                for (long long b = b0; b <= b1; ++b) list.push_back(v * p.B + (int)b);
            }
            off[(size_t)ty * gx + tx + 1] = (int)list.size();
        }
}

// Sweep tables of every ray (App. III Eq. A6 parametrisation; bin angles
// symmetric about the central ray, shifted by bin_offset), the count of
// nonzeros the kernels will meet, the per-tile ray lists of the
// backprojector and tan(beta_b) for the Eq. 11 backprojector.
void build_tables(const Plan& p, HostTables& t)
{
    t.ray.resize((size_t)p.V * p.B);
    t.range.resize((size_t)p.V * p.B);
    t.view.resize(p.V);
    t.view_d.resize(p.V);
    long long nnz = 0;
    for (int v = 0; v < p.V; ++v) {
        t.view[v] = make_float2((float)std::cos(p.angles[v]), (float)std::sin(p.angles[v]));
        t.view_d[v] = make_double2(std::cos(p.angles[v]), std::sin(p.angles[v]));
        for (int b = 0; b < p.B; ++b) {
            const double beta = ((double)b - 0.5 * (p.B - 1) + p.bin_offset) * p.dbeta;
            const HostRay R = make_ray(p, p.angles[v], beta);
            const size_t id = (size_t)v * p.B + b;
            t.ray[id] = R.fx();
            t.range[id] = make_int2(R.k_lo, R.k_hi);
            for_each_entry(R, p, [&](long long, float) { ++nnz; });
        }
    }
    t.nnz = nnz;
    bp_tile_lists(p, t.list_off, t.list);
    t.tau.resize((size_t)p.B + 2);
    for (int b = -1; b <= p.B; ++b) {
        const double beta = ((double)b - 0.5 * (p.B - 1) + p.bin_offset) * p.dbeta;
        t.tau[(size_t)b + 1] = std::tan(beta);  // |beta| < pi/2 by the geometry check
    }
}

void build_csr(const Plan& p, HostCsr& m)
{
    const int nrow = p.V * p.B;
    m.rowptr.assign((size_t)nrow + 1, 0);
    m.col.clear();
    m.val.clear();
    m.rows.clear();
    for (int v = 0; v < p.V; ++v)
        for (int b = 0; b < p.B; ++b) {
            const double beta = ((double)b - 0.5 * (p.B - 1) + p.bin_offset) * p.dbeta;
            const HostRay R = make_ray(p, p.angles[v], beta);
            for_each_entry(R, p, [&](long long pix, float c) {
                m.col.push_back((int)pix);
                m.val.push_back(c);
            });
            m.rows.push_back(R.rows ? 1 : 0);
            m.rowptr[(size_t)v * p.B + b + 1] = (long long)m.col.size();
        }
}

// The stored copies (see StoredMatrix): CSR by ray, chunked, with rays swept
// row by row indexing the transposed image; CSC by pixel, rays ascending.
int pack_stored(const Plan& p, HostStored& s)
{
    HostCsr m;
    build_csr(p, m);
    const long long nnz = (long long)m.col.size();
    if (nnz >= (1LL << 31) || (long long)p.nx * p.ny >= (1LL << 31)) return EPTV_ERR_ARG;
    const int nrow = p.V * p.B, npix = p.nx * p.ny;
    // the same entries grouped by pixel, rays ascending
    std::vector<long long> colcnt((size_t)npix + 1, 0);
    for (long long e = 0; e < nnz; ++e) colcnt[(size_t)m.col[e] + 1]++;
    for (int c = 0; c < npix; ++c) colcnt[(size_t)c + 1] += colcnt[c];
    std::vector<int> rowi((size_t)nnz);
    std::vector<float> cval((size_t)nnz);
    {
        std::vector<long long> fill(colcnt.begin(), colcnt.end() - 1);
        for (int r = 0; r < nrow; ++r)
            for (long long e = m.rowptr[r]; e < m.rowptr[r + 1]; ++e) {
                const long long at = fill[m.col[e]]++;
                rowi[at] = r;
                cval[at] = m.val[e];
            }
    }
    // padded, interleaved copies (see StoredMatrix)
    auto pack = [](int n, const long long* ptr, const int* idx, const float* val, bool chunked,
                   std::vector<int>& pptr, std::vector<int2>& ent) -> bool {
        pptr.assign((size_t)n + 1, 0);
        long long at = 0;
        for (int i = 0; i < n; ++i) {
            const long long len = ptr[i + 1] - ptr[i];
            at += (len + kStoredPad - 1) / kStoredPad * kStoredPad;
            if (at >= (1LL << 31)) return false;
            pptr[(size_t)i + 1] = (int)at;
        }
        ent.assign((size_t)at, int2{0, 0});
        for (int i = 0; i < n; ++i) {
            long long o = pptr[i];
            for (long long e = ptr[i]; e < ptr[i + 1]; ++e, ++o) {
                float v = val[e];
                int bits;
                std::memcpy(&bits, &v, 4);
                ent[(size_t)o] = int2{idx[e], bits};
            }
            for (; o < pptr[(size_t)i + 1]; ++o) ent[(size_t)o] = int2{idx[ptr[i + 1] - 1], 0};
            if (!chunked) continue;
            // chunks of kStoredChunk: slot l of a chunk of n holds entries l and n/2 + l
            for (long long c0 = pptr[i]; c0 < pptr[(size_t)i + 1]; c0 += kStoredChunk) {
                const long long nc = std::min<long long>(kStoredChunk, pptr[(size_t)i + 1] - c0), h = nc / 2;
                std::vector<int2> t(ent.begin() + c0, ent.begin() + c0 + nc);
                for (long long l = 0; l < h; ++l) {
                    ent[(size_t)(c0 + 2 * l)] = t[(size_t)l];
                    ent[(size_t)(c0 + 2 * l + 1)] = t[(size_t)(h + l)];
                }
            }
        }
        return true;
    };
    // the P copy: rays swept row by row index the transposed image
    std::vector<int> tcol(m.col);
    for (int r = 0; r < nrow; ++r)
        if (m.rows[r])
            for (long long e = m.rowptr[r]; e < m.rowptr[r + 1]; ++e)
                tcol[e] = (m.col[e] % p.nx) * p.ny + m.col[e] / p.nx;
    if (!pack(nrow, m.rowptr.data(), tcol.data(), m.val.data(), true, s.rowptr, s.rent) ||
        !pack(npix, colcnt.data(), rowi.data(), cval.data(), false, s.colptr, s.cent))
        return EPTV_ERR_ARG;
    s.nnz = nnz;
    s.rows = m.rows;
    // the compact encoding of the CSR copy (see StoredMatrix), when every
    // chunk's indices span at most 65535 and the words fit int32 offsets
    s.compact = true;
    s.rwordptr.assign((size_t)nrow + 1, 0);
    long long words = 0;
    for (int r = 0; r < nrow && s.compact; ++r) {
        const int n = s.rowptr[(size_t)r + 1] - s.rowptr[r];
        words += (long long)(n / kStoredChunk) * kChunkWords;
        if (n % kStoredChunk) words += 3 * (n % kStoredChunk) / 2 + 1;
        if (words >= (1LL << 31)) s.compact = false;
        s.rwordptr[(size_t)r + 1] = (int)words;
        for (int c0 = s.rowptr[r]; c0 < s.rowptr[(size_t)r + 1] && s.compact; c0 += kStoredChunk) {
            const int nc = std::min(kStoredChunk, s.rowptr[(size_t)r + 1] - c0);
            int lo = s.rent[(size_t)c0].x, hi = lo;
            for (int e = c0; e < c0 + nc; ++e) {
                lo = std::min(lo, s.rent[(size_t)e].x);
                hi = std::max(hi, s.rent[(size_t)e].x);
            }
            if (hi - lo > 0xffff) s.compact = false;
        }
    }
    if (!s.compact) {
        s.rwordptr.clear();
        return EPTV_OK;
    }
    s.rwords.assign((size_t)words, 0);
    for (int r = 0; r < nrow; ++r) {
        long long w = s.rwordptr[r];
        for (int c0 = s.rowptr[r]; c0 < s.rowptr[(size_t)r + 1]; c0 += kStoredChunk) {
            const int nc = std::min(kStoredChunk, s.rowptr[(size_t)r + 1] - c0), h = nc / 2;
            int base = s.rent[(size_t)c0].x;
            for (int e = c0; e < c0 + nc; ++e) base = std::min(base, s.rent[(size_t)e].x);
            for (int l = 0; l < h; ++l) {
                const int2 a = s.rent[(size_t)(c0 + 2 * l)], b = s.rent[(size_t)(c0 + 2 * l + 1)];
                s.rwords[(size_t)(w + 3 * l)] = a.y;
                s.rwords[(size_t)(w + 3 * l + 1)] = b.y;
                s.rwords[(size_t)(w + 3 * l + 2)] = (int)((unsigned)(a.x - base) | ((unsigned)(b.x - base) << 16));
            }
            s.rwords[(size_t)(w + 3 * h)] = base;
            w += 3 * h + 1;
        }
    }
    std::vector<int2>().swap(s.rent);
    return EPTV_OK;
}

}  // namespace eptv
