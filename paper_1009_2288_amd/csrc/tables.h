// tables.h -- host-only construction of everything a plan uploads: argument
// checks, the per-ray sweep tables, the backprojector's per-tile ray lists,
// the float32 system matrix (CSR by ray) and its padded stored copies.  No
// HIP runtime call is made here, so this code (with geometry.cpp) also builds
// with a plain host compiler, e.g. under the address and undefined-behaviour
// sanitizers.
#pragma once

#include <cstdint>
#include <vector>

#include "eptv_internal.h"

namespace eptv {

// Plan fields of a validated geometry (angles default to 2 pi v / V).
Plan host_plan(const eptv_geometry* g);
// EPTV_OK, or the status a bad geometry is rejected with.
int validate_geometry(const eptv_geometry* g);
int check_params(const eptv_params* q);
bool tv_eps_ok(double eps);
uint32_t select_rank(const Plan& p, double q);
float t0_of(const eptv_params& q);
float sigma_init(const eptv_params& q);
size_t n_edges(const Plan& p);

// Side of the backprojector's square pixel tiles.
constexpr int kBpTile = 16;

// Per tile, every ray that can meet one of its pixels (see tables.cpp).
void bp_tile_lists(const Plan& p, std::vector<int>& off, std::vector<int>& list);

// What plan creation uploads.
struct HostTables {
    std::vector<RayFx> ray;       // [V*B]
    std::vector<int2> range;      // [V*B]
    std::vector<float2> view;     // [V]
    std::vector<double2> view_d;  // [V]
    std::vector<double> tau;      // [B+2] tan of the bin angles, bins -1 .. B
    std::vector<int> list_off, list;
    long long nnz = 0;
};
void build_tables(const Plan& p, HostTables& t);

// The float32 system matrix of a plan, by ray (CSR): row v*B + b lists the
// pixels the ray meets with their lengths, in sweep order.
struct HostCsr {
    std::vector<long long> rowptr;
    std::vector<int> col;
    std::vector<float> val;
    std::vector<char> rows;  // per ray: swept row by row
};
void build_csr(const Plan& p, HostCsr& m);

// The padded, interleaved copies of StoredMatrix, as uploaded.
struct HostStored {
    std::vector<int> rowptr, colptr;  // entry offsets (padded) of the CSR and CSC copies
    std::vector<int2> rent, cent;     // wide CSR slots (emptied when compact), CSC pairs
    bool compact = false;             // the CSR copy is also held in the compact encoding:
    std::vector<int> rwordptr, rwords;  //  word offsets per ray and the chunks' words
    std::vector<char> rows;           // per ray: swept row by row (indexes the transposed image)
    long long nnz = 0;
};
// EPTV_OK, or EPTV_ERR_ARG when an index or offset would not fit int32.
int pack_stored(const Plan& p, HostStored& s);

}  // namespace eptv
