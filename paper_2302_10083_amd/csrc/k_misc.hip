// Small helper kernels: fills (used instead of memset so that every enqueued
// operation is a kernel node), the block state -> exact 3^n-bit repack, and a
// hash of words for comparing results.
#include "launch.h"
#include "h5.h"

namespace dqmc {

__global__ void fill_u64_kernel(uint64_t *p, uint64_t count, uint64_t value)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = value;
}

__global__ void fill_u32_kernel(uint32_t *p, uint64_t count, uint32_t value)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = value;
}

static uint32_t fill_grid(uint64_t count)
{
    uint64_t g = (count + 255) / 256;
    if (g > 4096) g = 4096;
    return (uint32_t)(g == 0 ? 1 : g);
}

hipError_t launch_fill_u64(uint64_t *p, uint64_t count, uint64_t value, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u64_kernel, dim3(fill_grid(count)), dim3(256), 0, s, p, count, value);
    return hipGetLastError();
}

hipError_t launch_fill_u32(uint32_t *p, uint64_t count, uint32_t value, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(fill_u32_kernel, dim3(fill_grid(count)), dim3(256), 0, s, p, count, value);
    return hipGetLastError();
}

// Output word j holds cubes 64j .. 64j+63.  Cube rho is bit rho % 243 of
// block rho / 243, i.e. bit (rho % 243) % 32 of logical word
// W = 8 * (rho / 243) + (rho % 243) / 32; with tile slots (padded) the word
// lies at (W / kTileWords) * kTileStride + W % kTileWords.  A run of cubes
// inside one word is copied at once.
__global__ void to_dense_kernel(const uint32_t *state, uint64_t *dense, uint64_t nwords, uint64_t ncubes,
                                int slots)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < nwords; j += stride) {
        uint64_t out = 0, r = 64 * j;
        const uint64_t rend = r + 64 < ncubes ? r + 64 : ncubes;
        uint32_t filled = 0;
        while (r < rend) {
            const uint64_t blk = r / kBlockCubes;
            const uint32_t p = (uint32_t)(r - blk * kBlockCubes), b = p & 31u;
            uint32_t take = 32u - b;
            if ((uint32_t)kBlockCubes - p < take) take = (uint32_t)kBlockCubes - p;
            if (rend - r < take) take = (uint32_t)(rend - r);
            const uint64_t W = kBlockWords * blk + (p >> 5);
            const uint64_t mem = slots ? (W / kTileWords) * kTileStride + W % kTileWords : W;
            const uint64_t bits = ((uint64_t)state[mem] >> b) & ((1ull << take) - 1ull);
            out |= bits << filled;
            filled += take;
            r += take;
        }
        dense[j] = out;
    }
}

hipError_t launch_to_dense(int n, const uint32_t *state, uint64_t *dense, hipStream_t s)
{
    const uint64_t ncubes = pow3(n), nwords = (ncubes + 63) / 64;
    hipLaunchKernelGGL(to_dense_kernel, dim3(fill_grid(nwords)), dim3(256), 0, s, state, dense, nwords, ncubes,
                       n > 12 ? 1 : 0);
    return hipGetLastError();
}

// Order-dependent hash: sum over i of a 64-bit mix of (i, word i), mod 2^64.
// The mix is the output finaliser of SplitMix64 (Steele, Lea and Flood,
// "Fast splittable pseudorandom number generators", OOPSLA 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__global__ void hash_kernel(const uint32_t *w, uint64_t n, unsigned long long *out)
{
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    uint64_t acc = 0;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        acc += mix64((i << 32) ^ (i >> 32) ^ ((uint64_t)w[i] * 0x9E3779B97F4A7C15ULL));
    acc = wave_sum(acc);
    if (lane_id() == 0) atomicAdd(out, (unsigned long long)acc);
}

hipError_t launch_hash(const uint32_t *w, uint64_t n, uint64_t *out, hipStream_t s)
{
    hipError_t e = launch_fill_u64(out, 1, 0, s);
    if (e != hipSuccess) return e;
    uint64_t g = (n + 255) / 256;
    if (g > 8192) g = 8192;
    hipLaunchKernelGGL(hash_kernel, dim3((uint32_t)(g == 0 ? 1 : g)), dim3(256), 0, s, w, n,
                       (unsigned long long *)out);
    return hipGetLastError();
}

}  // namespace dqmc
