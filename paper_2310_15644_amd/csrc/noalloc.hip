// efie_zx_flush64 for callers that cannot allocate device memory: the mixed
// solves' product (FP32 matrix cores, partial sums flushed into FP64) with its
// scratch in a static device array instead of a caller workspace.
#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "efie_internal.h"
#include "linalg.h"

// Scratch of the no-allocation variant: a file-scope device array, one copy per
// GPU the library runs on, held until the process ends.  Host code never passes
// its name to a kernel (on the host that name is only a stand-in); it takes the
// array's device address per device from hipGetSymbolAddress once, with that
// device current, and uses that address everywhere.
namespace {
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
__device__ __align__(256) char scratch[kNoAllocScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

__global__ void rows_iota_kernel(int* idx, int M) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < M; i += gridDim.x * blockDim.x) idx[i] = i;
}

void* scratch_for_current_device() {
    int dev = 0;
    EFIE_HIP_CHECK(hipGetDevice(&dev));
    EFIE_REQUIRE(dev >= 0 && dev < kMaxDevices, EFIE_ERR_STATE, "zx_flush64_noalloc: device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        EFIE_HIP_CHECK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        EFIE_REQUIRE(p != nullptr, EFIE_ERR_HIP, "zx_flush64_noalloc: no device address for the scratch array");
        g_scratch_ptr[dev] = p;
    }
    return g_scratch_ptr[dev];
}
}  // namespace

extern "C" int efie_zx_flush64_noalloc_max(int64_t* max_bytes) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(max_bytes != nullptr, EFIE_ERR_ARG, "zx_flush64_noalloc_max: null argument");
        *max_bytes = int64_t(kNoAllocScratchBytes);
        return int(EFIE_OK);
    });
}

extern "C" int efie_zx_flush64_noalloc(const void* Z, int64_t n, const void* X, void* Y, int64_t nrhs,
                                       hipStream_t stream) {
    return efie::guarded([&]() {
        EFIE_REQUIRE(Z && X && Y, EFIE_ERR_ARG, "zx_flush64_noalloc: null argument");
        EFIE_REQUIRE(n >= 1 && n < (int64_t(1) << 31) && nrhs >= 1 && nrhs < 65536, EFIE_ERR_ARG,
                     "zx_flush64_noalloc: bad sizes");
        const size_t xbytes = (size_t(n) * size_t(nrhs) * 8 + 255) & ~size_t(255);
        const size_t need = xbytes + size_t(nrhs) * sizeof(int);
        EFIE_REQUIRE(need <= kNoAllocScratchBytes, EFIE_ERR_ARG,
                     "zx_flush64_noalloc: n * nrhs * 8 bytes (rounded up to 256) + 4 nrhs exceed the " +
                         std::to_string(kNoAllocScratchBytes >> 20) + " MiB scratch; use efie_zx_flush64");
        char* ws = static_cast<char*>(scratch_for_current_device());
        float2* x32 = reinterpret_cast<float2*>(ws);
        int* idx = reinterpret_cast<int*>(ws + xbytes);
        // every scratch element the kernels read is written first in this call
        // (idx by rows_iota_kernel, x32 by gather_cast): nothing is carried over
        hipLaunchKernelGGL(rows_iota_kernel, dim3(int((nrhs + 255) / 256)), dim3(256), 0, stream, idx, int(nrhs));
        efie::gather_cast(static_cast<const double2*>(X), idx, int(nrhs), int(n), x32, stream);
        efie::cgemm_mfma_acc64(x32, Z, static_cast<double2*>(Y), idx, int(nrhs), int(n), stream);
        EFIE_HIP_CHECK(hipGetLastError());
        return int(EFIE_OK);
    });
}

