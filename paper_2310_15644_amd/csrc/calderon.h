// Internal declarations of the Calderon preconditioner (see calderon.cpp, calderon.hip).
#pragma once

#include "efie_internal.h"

struct efie_calderon_s {
    const efie_mesh_s* primal = nullptr;
    efie_mesh_s bary;                        // barycentric refinement (its own device tables)
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
    // device copies (caller-owned blob)
    void* dev = nullptr;
    std::vector<char> host_blob;             // sparse arrays packed for upload
    std::vector<size_t> offs;
    size_t bary_bytes = 0;                   // barycentric mesh tables at the start of the blob
};

namespace efie {
void build_calderon(efie_calderon_s& C, const efie_mesh_s& primal);
}  // namespace efie
