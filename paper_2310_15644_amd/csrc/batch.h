// Internal declarations of the batched (many-mesh) assembly and solve.
#pragma once

#include <vector>

#include "efie_internal.h"
#include "pair_kernels.h"

namespace efie {
struct BatchCol {           // COCG state of one mesh (one right-hand side)
    double rho_r, rho_i, bn2, rn2, tol2;
    int iters, status;
};
}  // namespace efie

struct efie_batch_s {
    std::vector<efie_mesh_s*> meshes;   // caller order
    std::vector<int> order;             // processing order (decreasing cost)
    std::vector<int64_t> zoff, voff;    // caller order: Z element offsets; vector offsets (n + 1)
    int64_t z_total = 0, v_total = 0;
    void* dev = nullptr;                // caller-owned device blob
    size_t off_zoff = 0, off_voff = 0;
    // the meshes' tables concatenated table by table in the blob (processing
    // order): cat points at them; per mesh (caller order) the triangles, RWGs,
    // ordered near pairs and those with q >= p of the meshes before it
    efie::DevMesh cat{};
    std::vector<int64_t> toff, noff, eoff, uoff;
};

namespace efie {
void batch_prepare(efie_batch_s& B);
void batch_cocg_init(const double2* b, double2* x, double2* r, double2* p, BatchCol* cols, int* active,
                     const int64_t* voff, int nm, double tol, hipStream_t s);
void batch_cocg_step(double2* x, double2* r, double2* p, const double2* q, BatchCol* cols, int* active,
                     const int64_t* voff, int nm, int* nact, hipStream_t s);
void batch_residual_norms(const double2* b, const double2* y, const int64_t* voff, int nm, double2* out,
                          hipStream_t s);
}  // namespace efie
