// Host-memory stand-ins for the HIP runtime calls that the plan builder makes,
// so that its validation, reordering and adjacency code can run under the
// address and undefined-behaviour sanitizers on a machine without a GPU.  Test
// infrastructure only: "device" buffers are plain host allocations, and an
// allocation can be made to fail after a set number of successes to drive the
// builder's clean-up paths.
#include <hip/hip_runtime_api.h>

#include <cstdlib>
#include <cstring>

namespace {
int g_fail_after = -1;   // < 0: never fail
int g_allocs = 0;

bool take() {
    if (g_fail_after >= 0 && g_allocs >= g_fail_after) return false;
    ++g_allocs;
    return true;
}
}  // namespace

extern "C" void stub_fail_after(int n) {
    g_fail_after = n;
    g_allocs = 0;
}
extern "C" int stub_allocations(void) { return g_allocs; }

hipError_t hipMalloc(void** ptr, size_t size) {
    if (!take()) return hipErrorOutOfMemory;
    *ptr = std::malloc(size ? size : 1);
    return *ptr ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* ptr) {
    std::free(ptr);
    return hipSuccess;
}
hipError_t hipHostMalloc(void** ptr, size_t size, unsigned int) {
    if (!take()) return hipErrorOutOfMemory;
    *ptr = std::malloc(size ? size : 1);
    return *ptr ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipHostFree(void* ptr) {
    std::free(ptr);
    return hipSuccess;
}
hipError_t hipHostGetDevicePointer(void** dev, void* host, unsigned int) {
    *dev = host;
    return hipSuccess;
}
hipError_t hipMemcpy(void* dst, const void* src, size_t n, hipMemcpyKind) {
    std::memmove(dst, src, n);
    return hipSuccess;
}
hipError_t hipMemset(void* dst, int value, size_t n) {
    std::memset(dst, value, n);
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t* ev, unsigned) {
    if (!take()) return hipErrorOutOfMemory;
    *ev = reinterpret_cast<hipEvent_t>(new char[16]);
    return hipSuccess;
}
hipError_t hipEventDestroy(hipEvent_t ev) {
    delete[] reinterpret_cast<char*>(ev);
    return hipSuccess;
}
hipError_t hipGetDevice(int* d) {
    *d = 0;
    return hipSuccess;
}
hipError_t hipDeviceSynchronize(void) { return hipSuccess; }
const char* hipGetErrorString(hipError_t) { return "stub error"; }
