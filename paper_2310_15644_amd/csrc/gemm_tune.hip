// The GEMM tile autotuner with a persistent cache of its choices on disk
// (efie_gemm_autotune_cached).  Built on the GEMM's own calls: the tile table
// (efie_gemm_variants / efie_gemm_variant_info), the timing of every tile
// (efie_gemm_autotune) and the selection (efie_gemm_select).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "efie_internal.h"

// ------------------------------------------------------- tile cache on disk
namespace efie {
// a seeded right-hand side block for timing: values in [-1, 1) from a 64-bit mix
__global__ void tune_fill_kernel(float2* x, size_t count) {
    for (size_t e = size_t(blockIdx.x) * blockDim.x + threadIdx.x; e < count; e += size_t(gridDim.x) * blockDim.x) {
        uint64_t h = (uint64_t(e) + 0x9e3779b97f4a7c15ull) * 0xbf58476d1ce4e5b9ull;
        h ^= h >> 31;
        h *= 0x94d049bb133111ebull;
        h ^= h >> 29;
        const float a = float(h & 0xffffff) * (2.0f / 16777216.0f) - 1.0f;
        const float b = float((h >> 32) & 0xffffff) * (2.0f / 16777216.0f) - 1.0f;
        x[e] = make_float2(a, b);
    }
}

namespace {
int num_variants() {
    int c = 0;
    EFIE_REQUIRE(efie_gemm_variants(&c) == EFIE_OK && c >= 1, EFIE_ERR_STATE, "autotune: no tile variants");
    return c;
}

size_t tune_x_bytes(int64_t n, int64_t M) { return (size_t(n) * size_t(M) * 8 + 255) & ~size_t(255); }

// key of a cache line: device, order, right-hand sides and the tile table, so a
// rebuilt library with other tiles never reuses a stale choice
std::string tune_key(int64_t n, int64_t M) {
    int dev = 0;
    EFIE_HIP_CHECK(hipGetDevice(&dev));
    hipDeviceProp_t prop{};
    EFIE_HIP_CHECK(hipGetDeviceProperties(&prop, dev));
    std::string name = std::string(prop.gcnArchName) + "/" + prop.name;
    for (char& c : name)
        if (c == ' ' || c == '\t' || c == '\n') c = '_';
    std::ostringstream k;
    k << name << "|n=" << n << "|M=" << M << "|tiles=";
    const int nv = num_variants();
    for (int v = 0; v < nv; ++v) {
        int bm = 0, bn = 0, kc = 0;
        EFIE_REQUIRE(efie_gemm_variant_info(v, &bm, &bn, &kc) == EFIE_OK, EFIE_ERR_STATE, "autotune: tile table");
        k << (v ? "," : "") << bm << "x" << bn << "x" << kc;
    }
    return k.str();
}

struct TuneEntry {
    int v32 = -1, v64 = -1;
    std::vector<double> ms32, ms64;
};

// one line per entry: <key> <v32> <v64> <ms32 x count> <ms64 x count>
bool parse_line(const std::string& line, int nv, std::string& key, TuneEntry& e) {
    std::istringstream in(line);
    if (!(in >> key >> e.v32 >> e.v64)) return false;
    e.ms32.assign(size_t(nv), 0.0);
    e.ms64.assign(size_t(nv), 0.0);
    for (int v = 0; v < nv; ++v)
        if (!(in >> e.ms32[size_t(v)])) return false;
    for (int v = 0; v < nv; ++v)
        if (!(in >> e.ms64[size_t(v)])) return false;
    return e.v32 >= 0 && e.v32 < nv && e.v64 >= 0 && e.v64 < nv;
}
}  // namespace
}  // namespace efie

extern "C" int efie_gemm_autotune_cached_workspace_size(int64_t n, int64_t M, size_t* bytes) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(bytes && n >= 1 && n < (int64_t(1) << 31) && M >= 1 && M < 65536, EFIE_ERR_ARG,
                     "gemm_autotune_cached_workspace_size: bad argument");
        *bytes = efie::tune_x_bytes(n, M) + ((size_t(M) * size_t(n) * 16 + 255) & ~size_t(255)) + size_t(M) * 4;
        return int(EFIE_OK);
    });
}

extern "C" int efie_gemm_autotune_cached(const char* cache_path, const void* Z, int64_t n, int64_t M, int reps,
                                         int force, void* ws, size_t ws_bytes, int* variant_acc32,
                                         int* variant_acc64, double* ms_acc32, double* ms_acc64, int* from_cache,
                                         hipStream_t stream) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(Z && ws && variant_acc32 && variant_acc64 && reps >= 1, EFIE_ERR_ARG,
                     "gemm_autotune_cached: bad argument");
        EFIE_REQUIRE(n >= 1 && n < (int64_t(1) << 31) && M >= 1 && M < 65536, EFIE_ERR_ARG,
                     "gemm_autotune_cached: bad sizes");
        size_t need = 0;
        EFIE_REQUIRE(efie_gemm_autotune_cached_workspace_size(n, M, &need) == EFIE_OK && ws_bytes >= need,
                     EFIE_ERR_ARG, "gemm_autotune_cached: workspace too small");
        EFIE_REQUIRE((reinterpret_cast<uintptr_t>(ws) & 255) == 0, EFIE_ERR_ARG,
                     "gemm_autotune_cached: workspace not 256-byte aligned");
        const int nv = efie::num_variants();
        const std::string key = efie::tune_key(n, M);
        std::vector<std::string> lines;
        efie::TuneEntry ent;
        bool hit = false;
        if (cache_path) {
            std::ifstream in(cache_path);
            std::string line;
            while (std::getline(in, line)) {
                std::string k;
                efie::TuneEntry e;
                if (!efie::parse_line(line, nv, k, e)) continue;   // malformed lines are dropped
                if (k == key) {
                    if (!force) {
                        ent = e;
                        hit = true;
                    }
                    continue;
                }
                lines.push_back(line);
            }
        }
        if (!hit) {
            char* base = static_cast<char*>(ws);
            float2* X = reinterpret_cast<float2*>(base);
            char* rest = base + efie::tune_x_bytes(n, M);
            const size_t count = size_t(n) * size_t(M);
            hipLaunchKernelGGL(efie::tune_fill_kernel, dim3(unsigned(std::min<size_t>((count + 255) / 256, 65536))),
                               dim3(256), 0, stream, X, count);
            EFIE_HIP_CHECK(hipGetLastError());
            ent.ms32.assign(size_t(nv), 0.0);
            ent.ms64.assign(size_t(nv), 0.0);
            const size_t rest_bytes = ws_bytes - efie::tune_x_bytes(n, M);
            int rc = efie_gemm_autotune(Z, n, X, M, 0, rest, rest_bytes, reps, ent.ms32.data(), &ent.v32, stream);
            if (rc != EFIE_OK) return rc;
            rc = efie_gemm_autotune(Z, n, X, M, 1, rest, rest_bytes, reps, ent.ms64.data(), &ent.v64, stream);
            if (rc != EFIE_OK) return rc;
            efie::clear_error();
            if (cache_path) {
                std::ostringstream l;
                l << key << " " << ent.v32 << " " << ent.v64;
                l.precision(17);   // round trip: a reused entry returns the same doubles
                for (double x : ent.ms32) l << " " << x;
                for (double x : ent.ms64) l << " " << x;
                lines.push_back(l.str());
                // written to a temporary file and renamed, so readers never see half a file;
                // an unwritable cache leaves the timing result valid (no error)
                const std::string tmp = std::string(cache_path) + ".tmp";
                {
                    std::ofstream out(tmp, std::ios::trunc);
                    for (const auto& s : lines) out << s << "\n";
                }
                std::rename(tmp.c_str(), cache_path);
            }
        }
        EFIE_REQUIRE(efie_gemm_select(0, ent.v32, nullptr) == EFIE_OK && efie_gemm_select(1, ent.v64, nullptr) == EFIE_OK,
                     EFIE_ERR_STATE, "gemm_autotune_cached: selection failed");
        *variant_acc32 = ent.v32;
        *variant_acc64 = ent.v64;
        for (int v = 0; v < nv; ++v) {
            if (ms_acc32) ms_acc32[v] = ent.ms32[size_t(v)];
            if (ms_acc64) ms_acc64[v] = ent.ms64[size_t(v)];
        }
        if (from_cache) *from_cache = hit ? 1 : 0;
        return int(EFIE_OK);
    });
}

