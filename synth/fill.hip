// Device twin of synth/inputs.py: the counter-based generator of uniform
// Goldilocks words (SplitMix64 finaliser, Steele, Lea and Flood, OOPSLA 2014),
// used to fill large inputs directly in device memory.  It draws numbers only;
// the single comparison with p is rejection sampling.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

namespace {
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kP = 0xFFFFFFFF00000001ull;

__device__ __forceinline__ uint64_t mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ void k_fill(uint64_t *out, size_t count, uint64_t key, uint64_t start) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (size_t)gridDim.x * blockDim.x) {
        uint64_t z = mix(key + (start + i + 1) * kGamma);
        while (z >= kP) z = mix(z + kGamma);
        out[i] = z;
    }
}
}  // namespace

// Writes words start .. start+count-1 of the stream with the given key
// (key = stream_key(seed, stream) from synth/inputs.py) to dev_out.
// Returns 0, or -1 for a bad argument, -3 for a HIP error.
extern "C" int synth_fill_goldilocks(uint64_t *dev_out, size_t count, uint64_t key, uint64_t start, void *stream) {
    if (dev_out == nullptr || count == 0) return -1;
    hipDeviceptr_t base = nullptr;
    size_t size = 0;
    if (hipMemGetAddressRange(&base, &size, (hipDeviceptr_t)dev_out) == hipSuccess && base != nullptr) {
        size_t off = (size_t)((char *)dev_out - (char *)base);
        if (off > size || count > (size - off) / sizeof(uint64_t)) return -1;
    } else {
        (void)hipGetLastError();
        return -1;
    }
    size_t blocks = (count + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    hipLaunchKernelGGL(k_fill, dim3((unsigned)blocks), dim3(256), 0, (hipStream_t)stream, dev_out, count, key, start);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}
