// C ABI entry points for mesh handles, errors and versioning.
#include <cmath>
#include <cstring>

#include "efie_internal.h"

namespace efie {
namespace {
thread_local std::string g_last_error;
}
void set_error(const std::string& msg) { g_last_error = msg; }
void clear_error() { g_last_error.clear(); }
}  // namespace efie

using efie::guarded;

extern "C" {

int efie_abi_version(void) { return EFIE_ABI_VERSION; }

const char* efie_last_error(void) { return efie::g_last_error.c_str(); }

int efie_mesh_create(const double* xyz, int64_t nv, const int32_t* tri, int64_t nt, double near_factor,
                     efie_mesh* out) {
    return guarded([&]() {
        EFIE_REQUIRE(out != nullptr, EFIE_ERR_ARG, "mesh_create: out is null");
        auto* m = new efie_mesh_s();
        try {
            efie::build_mesh(*m, xyz, nv, tri, nt, near_factor);
            efie::pack_tables(*m);
        } catch (...) {
            delete m;
            throw;
        }
        *out = m;
        return int(EFIE_OK);
    });
}

void efie_mesh_destroy(efie_mesh mesh) { delete mesh; }

int efie_mesh_set_far_rule(efie_mesh mesh, double ratio) {
    return guarded([&]() {
        EFIE_REQUIRE(mesh != nullptr, EFIE_ERR_ARG, "mesh_set_far_rule: null mesh");
        EFIE_REQUIRE(std::isfinite(ratio) && ratio >= 0.0, EFIE_ERR_ARG, "mesh_set_far_rule: ratio must be >= 0");
        mesh->far3 = ratio;
        mesh->dm.far3 = ratio;   // the device view (taken by value at each launch)
        return int(EFIE_OK);
    });
}

int efie_mesh_fp32_kmax(efie_mesh mesh, double* kmax) {
    return guarded([&]() {
        EFIE_REQUIRE(mesh != nullptr && kmax != nullptr, EFIE_ERR_ARG, "mesh_fp32_kmax: null argument");
        *kmax = efie::fp32_kmax(mesh->diam);
        return int(EFIE_OK);
    });
}

int efie_ktilde(double k, double a, double* kt_re, double* kt_im) {
    return guarded([&]() {
        EFIE_REQUIRE(kt_re != nullptr && kt_im != nullptr, EFIE_ERR_ARG, "ktilde: null output");
        EFIE_REQUIRE(std::isfinite(k) && k > 0.0 && std::isfinite(a) && a > 0.0, EFIE_ERR_ARG,
                     "ktilde: need finite k > 0 and a > 0");
        *kt_re = k;
        *kt_im = -0.4 * std::cbrt(k) / std::cbrt(a * a);
        return int(EFIE_OK);
    });
}

int efie_mesh_sizes(efie_mesh mesh, int64_t* n_rwg, int64_t* n_tri, int64_t* n_near, size_t* table_bytes) {
    return guarded([&]() {
        EFIE_REQUIRE(mesh != nullptr, EFIE_ERR_ARG, "mesh_sizes: null mesh");
        if (n_rwg) *n_rwg = mesh->N;
        if (n_tri) *n_tri = mesh->T;
        if (n_near) *n_near = int64_t(mesh->near_p.size());
        if (table_bytes) *table_bytes = mesh->host_blob.size();
        return int(EFIE_OK);
    });
}

int efie_mesh_rwg_table(efie_mesh mesh, int32_t* edge_v, int32_t* edge_t) {
    return guarded([&]() {
        EFIE_REQUIRE(mesh != nullptr, EFIE_ERR_ARG, "mesh_rwg_table: null mesh");
        if (edge_v) std::memcpy(edge_v, mesh->edge_v.data(), mesh->edge_v.size() * sizeof(int32_t));
        if (edge_t) std::memcpy(edge_t, mesh->edge_t.data(), mesh->edge_t.size() * sizeof(int32_t));
        return int(EFIE_OK);
    });
}

int efie_mesh_upload(efie_mesh mesh, void* dev, size_t bytes, hipStream_t stream) {
    return guarded([&]() {
        EFIE_REQUIRE(mesh != nullptr && dev != nullptr, EFIE_ERR_ARG, "mesh_upload: null argument");
        EFIE_REQUIRE(bytes >= mesh->host_blob.size(), EFIE_ERR_ARG, "mesh_upload: buffer too small");
        EFIE_REQUIRE((reinterpret_cast<uintptr_t>(dev) & 255) == 0, EFIE_ERR_ARG,
                     "mesh_upload: device buffer must be 256-byte aligned");
        EFIE_HIP_CHECK(hipMemcpyAsync(dev, mesh->host_blob.data(), mesh->host_blob.size(),
                                      hipMemcpyHostToDevice, stream));
        EFIE_HIP_CHECK(hipStreamSynchronize(stream));
        efie::bind_tables(*mesh, dev);
        mesh->dev_bytes = bytes;
        return int(EFIE_OK);
    });
}

}  // extern "C"
