// Internal declarations of the Calderon preconditioner (see calderon.cpp, calderon.hip).
#pragma once

#include "efie_internal.h"

struct efie_calderon_s {
    const efie_mesh_s* primal = nullptr;
    efie_mesh_s bary;                        // barycentric refinement (its own device tables)
    double far3 = -1.0;                      // far rule of the barycentric operator (< 0: the primal's)
    int64_t N = 0;
    // R: Buffa-Christiansen coefficients, CSC by BC function n (rows: barycentric RWGs)
    std::vector<int32_t> r_ptr, r_idx;
    std::vector<double> r_val;
    // the same entries by barycentric RWG (CSR of R)
    std::vector<int32_t> re_ptr, re_idx;
    std::vector<double> re_val;
    // mixed Gram matrix G (CSR by primal RWG m) and its transpose
    std::vector<int32_t> g_ptr, g_idx, gt_ptr, gt_idx;
    std::vector<double> g_val, gt_val;
    std::vector<int32_t> n_order;            // primal RWGs in a spatially coherent (Morton) order
    std::vector<int32_t> bary_canon;         // canonical index of each barycentric RWG
    std::vector<int8_t> bary_flip;           // 1 where the canonical RWG is the internal one negated
    // runs of at most BC_BLOCK consecutive BC functions in n_order (first position
    // run_t0), the distinct barycentric RWGs each run reads (CSR u_ptr / u_idx,
    // sorted, at most BC_UMAX) and, per entry of R's CSC, the local position of its
    // RWG in the run's list
    std::vector<int32_t> run_t0, u_ptr, u_idx, r_loc;
    int64_t u_max = 0;
    // device copies (caller-owned blob)
    void* dev = nullptr;
    std::vector<char> host_blob;             // sparse arrays packed for upload
    std::vector<size_t> offs;
    size_t bary_bytes = 0;                   // barycentric mesh tables at the start of the blob
};

namespace efie {
constexpr int BC_BLOCK = 256;   // BC functions per block of the source-side contraction
// distinct barycentric RWGs per block (its LDS list): a run closes when its next
// BC function would exceed it, so at level 5 runs hold about 140 functions
constexpr int BC_UMAX = 1024;
bool verbose();
void build_calderon(efie_calderon_s& C, const efie_mesh_s& primal);
}  // namespace efie
