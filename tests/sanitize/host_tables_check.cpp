// Host-side plan construction of libeptv, built with the address and
// undefined-behaviour sanitizers by tests/test_host_sanitizers.py and run on
// the CPU (no HIP runtime call is involved).  Besides running every table
// builder under the sanitizers it checks the invariants the kernels rely on:
//  * the nonzero count of the sweep tables equals the CSR's;
//  * every (ray, pixel) entry of the matrix has its ray in the backprojector's
//    list for the pixel's tile (otherwise P^T would drop that entry);
//  * the stored copies are padded to whole 4-entry groups, the CSR chunks
//    un-interleave to the ray's entries (transposed index for row sweeps) and
//    the CSC holds the same entries regrouped by pixel, rays ascending;
//  * bad geometries and parameters are rejected.
// Exit status 0 on success; a sanitizer report aborts with a non-zero status.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <utility>
#include <vector>

#include "tables.h"

using namespace eptv;

static int g_fail = 0;
#define CHECK(cond, ...)                                  \
    do {                                                  \
        if (!(cond)) {                                    \
            std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
            std::fprintf(stderr, __VA_ARGS__);            \
            std::fprintf(stderr, "\n");                   \
            ++g_fail;                                     \
        }                                                 \
    } while (0)

static eptv_geometry geom(int nx, int ny, double pix, int V, int B, double sad, double sdd, double offset,
                          const double* angles = nullptr)
{
    eptv_geometry g{};
    g.nx = nx;
    g.ny = ny;
    g.pixel_mm = pix;
    g.n_views = V;
    g.view_angles_rad = angles;
    g.n_bins = B;
    // the fan just covers the image's half-diagonal
    const double r = 0.5 * pix * std::sqrt((double)nx * nx + (double)ny * ny);
    g.dbeta_rad = 2.0 * std::asin(r / sad) / B;
    g.bin_offset = offset;
    g.sad_mm = sad;
    g.sdd_mm = sdd;
    return g;
}

static void check_geometry(const eptv_geometry& g, const char* name, int want_compact = -1)
{
    CHECK(validate_geometry(&g) == EPTV_OK, "%s: geometry rejected", name);
    const Plan p = host_plan(&g);
    HostTables t;
    build_tables(p, t);
    HostCsr m;
    build_csr(p, m);
    const int nrow = p.V * p.B, npix = p.nx * p.ny;
    CHECK((long long)m.col.size() == t.nnz, "%s: nnz %lld vs %zu", name, t.nnz, m.col.size());
    CHECK((int)m.rowptr.size() == nrow + 1 && m.rowptr[0] == 0, "%s: rowptr", name);
    for (size_t e = 0; e < m.col.size(); ++e) {
        CHECK(m.col[e] >= 0 && m.col[e] < npix, "%s: column %d", name, m.col[e]);
        CHECK(m.val[e] > 0.0f && m.val[e] <= 1.5f * (float)p.pixel, "%s: length %g", name, (double)m.val[e]);
    }
    // tile lists cover every entry
    const int gx = (p.nx + kBpTile - 1) / kBpTile, gy = (p.ny + kBpTile - 1) / kBpTile;
    CHECK((int)t.list_off.size() == gx * gy + 1, "%s: list offsets", name);
    std::vector<std::vector<char>> in_list((size_t)gx * gy);
    for (int tile = 0; tile < gx * gy; ++tile) {
        CHECK(t.list_off[tile] <= t.list_off[tile + 1], "%s: list offsets decrease", name);
        in_list[tile].assign((size_t)nrow, 0);
        int prev = -1;
        for (int k = t.list_off[tile]; k < t.list_off[tile + 1]; ++k) {
            const int id = t.list[(size_t)k];
            CHECK(id >= 0 && id < nrow, "%s: ray id %d", name, id);
            CHECK(id > prev, "%s: list not ascending", name);
            prev = id;
            if (id >= 0 && id < nrow) in_list[tile][(size_t)id] = 1;
        }
    }
    long long missing = 0;
    for (int r = 0; r < nrow; ++r)
        for (long long e = m.rowptr[r]; e < m.rowptr[r + 1]; ++e) {
            const int i = m.col[e] % p.nx, j = m.col[e] / p.nx;
            const int tile = (j / kBpTile) * gx + i / kBpTile;
            if (!in_list[tile][(size_t)r]) ++missing;
        }
    CHECK(missing == 0, "%s: %lld entries whose ray is not in their tile's list", name, missing);
    CHECK((int)t.tau.size() == p.B + 2, "%s: tau", name);
    for (double v : t.tau) CHECK(std::isfinite(v), "%s: tau not finite", name);

    // stored copies
    HostStored s;
    CHECK(pack_stored(p, s) == EPTV_OK, "%s: pack_stored", name);
    CHECK(s.nnz == t.nnz, "%s: stored nnz", name);
    CHECK(s.rows == m.rows, "%s: stored row-sweep flags", name);
    CHECK(want_compact < 0 || (int)s.compact == want_compact, "%s: CSR encoding compact = %d", name, (int)s.compact);
    CHECK(s.compact ? s.rent.empty() && (int)s.rwordptr.size() == nrow + 1 : s.rwords.empty(), "%s: one CSR encoding",
          name);
    CHECK((int)s.rowptr.size() == nrow + 1 && (int)s.colptr.size() == npix + 1, "%s: stored offsets", name);
    for (int r = 0; r < nrow; ++r) {
        const int a = s.rowptr[r], b = s.rowptr[r + 1];
        const long long len = m.rowptr[r + 1] - m.rowptr[r];
        CHECK(a % kStoredPad == 0 && b % kStoredPad == 0, "%s: row %d not padded", name, r);
        CHECK(b - a == (len + kStoredPad - 1) / kStoredPad * kStoredPad, "%s: row %d padded length", name, r);
        // un-interleave the chunks: slot l of a chunk of n holds entries l and n/2 + l;
        // compact slots are (length bits, length bits, 16-bit offsets) and the chunk's base
        std::vector<int2> flat((size_t)(b - a));
        long long wpos = s.compact ? s.rwordptr[(size_t)r] : 0;
        for (int c0 = a; c0 < b; c0 += kStoredChunk) {
            const int nc = std::min(kStoredChunk, b - c0), h = nc / 2;
            for (int l = 0; l < h; ++l) {
                if (s.compact) {
                    const int base = s.rwords[(size_t)(wpos + 3 * h)];
                    const unsigned off = (unsigned)s.rwords[(size_t)(wpos + 3 * l + 2)];
                    flat[(size_t)(c0 - a + l)] = int2{base + (int)(off & 0xffffu), s.rwords[(size_t)(wpos + 3 * l)]};
                    flat[(size_t)(c0 - a + h + l)] = int2{base + (int)(off >> 16), s.rwords[(size_t)(wpos + 3 * l + 1)]};
                } else {
                    flat[(size_t)(c0 - a + l)] = s.rent[(size_t)(c0 + 2 * l)];
                    flat[(size_t)(c0 - a + h + l)] = s.rent[(size_t)(c0 + 2 * l + 1)];
                }
            }
            wpos += 3 * h + 1;
        }
        if (s.compact) CHECK(wpos == s.rwordptr[(size_t)r + 1], "%s: row %d compact words", name, r);
        for (long long e = 0; e < len; ++e) {
            const int col = m.col[m.rowptr[r] + e];
            const int want = m.rows[r] ? (col % p.nx) * p.ny + col / p.nx : col;
            float got;
            std::memcpy(&got, &flat[(size_t)e].y, 4);
            CHECK(flat[(size_t)e].x == want && got == m.val[m.rowptr[r] + e], "%s: stored row %d entry %lld", name,
                  r, e);
        }
        for (long long e = len; e < b - a; ++e) CHECK(flat[(size_t)e].y == 0, "%s: padding length", name);
    }
    std::map<std::pair<int, int>, float> by_pixel;
    for (int r = 0; r < nrow; ++r)
        for (long long e = m.rowptr[r]; e < m.rowptr[r + 1]; ++e) by_pixel[{m.col[e], r}] = m.val[e];
    long long seen = 0;
    for (int c = 0; c < npix; ++c) {
        CHECK(s.colptr[c] % kStoredPad == 0, "%s: column %d not padded", name, c);
        int prev = -1;
        for (int e = s.colptr[c]; e < s.colptr[c + 1]; ++e) {
            float v;
            std::memcpy(&v, &s.cent[(size_t)e].y, 4);
            if (v == 0.0f) continue;  // padding
            const int r = s.cent[(size_t)e].x;
            CHECK(r > prev, "%s: column %d rays not ascending", name, c);
            prev = r;
            auto it = by_pixel.find({c, r});
            CHECK(it != by_pixel.end() && it->second == v, "%s: CSC entry (%d, %d)", name, c, r);
            ++seen;
        }
    }
    CHECK(seen == t.nnz, "%s: CSC holds %lld of %lld entries", name, seen, t.nnz);
    std::printf("%s: %d x %d, %d x %d, nnz %lld, list %zu ids, stored %s CSR (%zu slots / %zu words) + %zu CSC\n",
                name, p.nx, p.ny, p.V, p.B, t.nnz, t.list.size(), s.compact ? "compact" : "wide", s.rent.size(),
                s.rwords.size(), s.cent.size());
}

static void check_rejections()
{
    eptv_geometry g = geom(16, 16, 1.0, 8, 32, 100.0, 200.0, 0.0);
    CHECK(validate_geometry(nullptr) == EPTV_ERR_ARG, "null geometry");
    eptv_geometry b = g;
    b.nx = 1;
    CHECK(validate_geometry(&b) == EPTV_ERR_ARG, "1-pixel-wide image");
    b = g;
    b.n_bins = 0;
    CHECK(validate_geometry(&b) == EPTV_ERR_ARG, "no bins");
    b = g;
    b.sad_mm = 10.0;  // inside the image
    CHECK(validate_geometry(&b) == EPTV_ERR_GEOMETRY, "source inside the image");
    b = g;
    b.dbeta_rad = -1e-3;
    CHECK(validate_geometry(&b) == EPTV_ERR_GEOMETRY, "negative bin pitch");
    b = g;
    b.pixel_mm = NAN;
    CHECK(validate_geometry(&b) == EPTV_ERR_GEOMETRY, "NaN pixel");
    b = g;
    b.sdd_mm = 50.0;
    CHECK(validate_geometry(&b) == EPTV_ERR_GEOMETRY, "detector nearer than the source distance");
    b = g;
    b.dbeta_rad = 0.1;  // fan wider than a half-plane
    CHECK(validate_geometry(&b) == EPTV_ERR_GEOMETRY, "fan too wide");
    double ang[8] = {0, 1, 2, 3, NAN, 5, 6, 7};
    b = g;
    b.view_angles_rad = ang;
    CHECK(validate_geometry(&b) == EPTV_ERR_GEOMETRY, "NaN view angle");

    eptv_params q{};
    q.outer_iters = 3;
    q.cgls_iters = 3;
    q.tv_iters = 5;
    q.zero_init = 1;
    q.mu = 1.0;
    q.lambda = 1000.0;
    q.edge_quantile = 0.9;
    q.sigma_fixed = -1.0;
    q.sigma_floor = 1e-12;
    q.tv_eps = 1e-4;
    q.armijo_c = 1e-4;
    q.armijo_shrink = 0.5;
    q.armijo_max_backtracks = 20;
    q.positivity = 1;
    CHECK(check_params(&q) == EPTV_OK, "default parameters rejected");
    eptv_params r = q;
    r.tv_eps = 0.0;
    CHECK(check_params(&r) == EPTV_ERR_ARG, "eps 0 accepted");
    r = q;
    r.tv_eps = 1e-30;  // its float square underflows
    CHECK(check_params(&r) == EPTV_ERR_ARG, "eps with a zero float square accepted");
    r = q;
    r.cgls_iters = kMaxCgls + 1;
    CHECK(check_params(&r) == EPTV_ERR_ARG, "too many CGLS steps accepted");
    r = q;
    r.armijo_shrink = 1.0;
    CHECK(check_params(&r) == EPTV_ERR_ARG, "shrink 1 accepted");
    r = q;
    r.edge_quantile = 0.0;
    CHECK(check_params(&r) == EPTV_ERR_ARG, "quantile 0 accepted");
    r = q;
    r.stop_rmse = NAN;
    CHECK(check_params(&r) == EPTV_ERR_ARG, "NaN stop_rmse accepted");
    r = q;
    r.stored_matrix = 3;
    CHECK(check_params(&r) == EPTV_ERR_ARG, "operator mode 3 accepted");
    CHECK(check_params(nullptr) == EPTV_ERR_ARG, "null parameters accepted");

    const Plan p = host_plan(&g);
    CHECK(select_rank(p, 1.0) == (uint32_t)(n_edges(p) - 1), "rank at q = 1");
    CHECK(select_rank(p, 1e-12) == 0, "rank at a tiny q");
    CHECK(t0_of(q) == (float)(1.0 / 1000.0), "default first step");
}

int main()
{
    check_rejections();
    // small and odd shapes, a grid-line ray (odd bin count), an offset
    // detector, given view angles, and the small workload at full size
    const double ang[5] = {0.0, 0.7853981633974483, 1.5707963267948966, 2.5, 4.0};
    check_geometry(geom(8, 8, 1.0, 6, 24, 40.0, 80.0, 0.0), "8x8");
    check_geometry(geom(5, 7, 1.0, 7, 13, 30.0, 60.0, 0.0), "5x7 odd bins");
    check_geometry(geom(2, 2, 0.5, 4, 5, 10.0, 20.0, 0.0), "2x2");
    check_geometry(geom(77, 53, 1.1, 13, 101, 300.0, 600.0, 0.3), "77x53 offset");
    check_geometry(geom(33, 18, 0.9, 5, 64, 80.0, 160.0, -0.45, ang), "33x18 given angles");
    check_geometry(geom(65, 65, 1.0, 7, 129, 400.0, 800.0, 0.0), "65x65 isocentre ray");
    check_geometry(geom(128, 128, 1.0, 30, 256, 500.0, 1000.0, 0.0), "128x128 30 views", 1);
    // a 1100-pixel-wide image seen at 45 degrees: a 128-entry chunk of a
    // diagonal ray spans ~64 image rows (> 65535 indices), so the CSR copy
    // keeps the wide encoding
    check_geometry(geom(1100, 1100, 0.5, 2, 64, 2000.0, 4000.0, 0.0, ang), "1100x1100 wide CSR", 0);
    if (g_fail) {
        std::fprintf(stderr, "%d checks failed\n", g_fail);
        return 1;
    }
    std::printf("host tables: all checks passed\n");
    return 0;
}
