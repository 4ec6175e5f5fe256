// Device helpers shared by the kernel files (wavefront = 64 lanes on CDNA4).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fsv {

constexpr int kMaxGrid = 8192;
constexpr int kWave = 64;

static __device__ __forceinline__ int popc(uint64_t v) { return __popcll(v); }
static __device__ __forceinline__ int popc(uint32_t v) { return __popc(v); }

static __device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Block-wide ordered sum; every thread gets the result.  At most 1024 threads
// (1-, 2- or 3-D).  Deterministic: wavefront butterflies, then the wave sums
// in wave order.
static __device__ double block_sum(double v) {
    __shared__ double red[1024 / kWave];
    const int tid = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    const int nthr = blockDim.x * blockDim.y * blockDim.z;
    const int lane = tid % kWave, wid = tid / kWave;
    const int nw = (nthr + kWave - 1) / kWave;
    v = wave_sum(v);
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w];
    __syncthreads();
    return s;
}

static inline unsigned blocks_for(int64_t n, int block) {
    int64_t b = (n + block - 1) / block;
    if (b < 1) b = 1;
    if (b > kMaxGrid) b = kMaxGrid;
    return (unsigned)b;
}

}  // namespace fsv
