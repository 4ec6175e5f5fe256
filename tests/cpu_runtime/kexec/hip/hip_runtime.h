// CPU execution of the library's kernels (test infrastructure).
//
// Replaces <hip/hip_runtime.h> when the library's sources are compiled as
// plain C++ for the host: kernels become ordinary functions, and a launch
// runs them in the host stand-in (hip_stub.cpp), one fiber per work-item,
// one workgroup after another, with workgroup barriers, wavefront exchanges
// (shuffles, DPP moves, the FP64 matrix instruction) and dynamic LDS
// emulated there.  With AddressSanitizer every access a kernel
// makes to an allocation, a static array or its dynamic LDS is checked.
#pragma once

#include <hip/hip_runtime_api.h>
#include <hip/hip_vector_types.h>
#include <stdint.h>

#include <cmath>
#include <cstring>
#include <tuple>
#include <type_traits>
#include <utility>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __launch_bounds__(...)
#define __shared__ static
#define __align__(n) __attribute__((aligned(n)))

struct fsv_cpu_idx {
    uint32_t x, y, z;
};
extern thread_local fsv_cpu_idx threadIdx, blockIdx;
extern thread_local dim3 blockDim, gridDim;

// ---- provided by the host stand-in ----
void *fsv_cpu_dyn_lds();
void fsv_cpu_syncthreads();
// Wavefront exchange: this lane publishes n bytes; after every live lane of
// the wavefront has published, out receives the bytes lane src published.
void fsv_cpu_wave_exchange(const void *mine, void *out, size_t n, int src);
// Wavefront-wide 16x16x4 FP64 matrix product (operand layout of the hardware
// instruction: lane l holds A[l % 16][l / 16], B[l / 16][l % 16] and
// D[4 r + l / 16][l % 16], r = 0..3).
void fsv_cpu_mfma_f64_16x16x4(double a, double b, const double *c, double *d);
hipError_t fsv_cpu_launch(const void *fn, const char *name, dim3 g, dim3 b, size_t shm, hipStream_t st,
                          hipEvent_t e0, hipEvent_t e1, void (*run)(void *), void *ctx, void (*del)(void *),
                          void *(*copy)(void *));
const void *fsv_cpu_symbol(const void *p, size_t n);
void fsv_cpu_enable();
static const int fsv_cpu_enabled = (fsv_cpu_enable(), 0);  // kernels are known by address from now on

inline int fsv_cpu_lane() {
    const uint32_t t = threadIdx.x + blockDim.x * (threadIdx.y + blockDim.y * threadIdx.z);
    return (int)(t % 64u);
}

template <typename T>
inline T __shfl_xor(T v, int mask, int width = 64) {
    const int l = fsv_cpu_lane();
    const int src = (l & ~(width - 1)) | ((l ^ mask) & (width - 1));
    T out;
    fsv_cpu_wave_exchange(&v, &out, sizeof(T), src);
    return out;
}

// DPP lane move of a 32-bit value (quad permutations, row shifts, mirrors and
// broadcasts); lanes whose source is invalid or whose row is masked off get old.
inline int fsv_cpu_update_dpp(int old, int src, int ctrl, int row_mask, int bank_mask, bool bound_ctrl) {
    const int l = fsv_cpu_lane(), row = l >> 4, r = l & 15;
    int from = -1;
    if (ctrl <= 0xFF) {
        from = (l & ~3) | ((ctrl >> (2 * (l & 3))) & 3);
    } else if (ctrl >= 0x101 && ctrl <= 0x10F) {  // row_shl
        const int s = ctrl & 15;
        from = r + s < 16 ? l + s : -1;
    } else if (ctrl >= 0x111 && ctrl <= 0x11F) {  // row_shr
        const int s = ctrl & 15;
        from = r - s >= 0 ? l - s : -1;
    } else if (ctrl >= 0x121 && ctrl <= 0x12F) {  // row_ror
        from = (row << 4) | ((r + (ctrl & 15)) & 15);
    } else if (ctrl == 0x140) {  // row_mirror
        from = (row << 4) | (15 - r);
    } else if (ctrl == 0x141) {  // row_half_mirror
        from = (row << 4) | ((r & 8) | (7 - (r & 7)));
    } else if (ctrl == 0x142) {  // row_bcast15
        from = row > 0 ? ((row - 1) << 4) | 15 : -1;
    } else if (ctrl == 0x143) {  // row_bcast31
        from = row > 1 ? 31 : -1;
    } else {
        std::abort();  // a control the emulation does not know
    }
    int got = 0;
    fsv_cpu_wave_exchange(&src, &got, sizeof(int), from < 0 ? l : from);
    const bool row_on = (row_mask >> row) & 1, bank_on = (bank_mask >> ((l >> 2) & 3)) & 1;
    if (!row_on || !bank_on) return old;
    if (from < 0) return bound_ctrl ? 0 : old;
    return got;
}
#define __builtin_amdgcn_update_dpp fsv_cpu_update_dpp
#define __builtin_amdgcn_readfirstlane(x) (x)

typedef double fsv_cpu_double4 __attribute__((ext_vector_type(4)));
inline fsv_cpu_double4 fsv_cpu_mfma(double a, double b, fsv_cpu_double4 c, int, int, int) {
    double ci[4] = {c[0], c[1], c[2], c[3]}, d[4];
    fsv_cpu_mfma_f64_16x16x4(a, b, ci, d);
    return fsv_cpu_double4{d[0], d[1], d[2], d[3]};
}
#define __builtin_amdgcn_mfma_f64_16x16x4f64 fsv_cpu_mfma

inline int __popc(uint32_t v) { return __builtin_popcount(v); }
inline int __popcll(uint64_t v) { return __builtin_popcountll(v); }
inline int __double2loint(double d) {
    uint64_t u;
    std::memcpy(&u, &d, 8);
    return (int)(uint32_t)u;
}
inline int __double2hiint(double d) {
    uint64_t u;
    std::memcpy(&u, &d, 8);
    return (int)(uint32_t)(u >> 32);
}
inline double __hiloint2double(int hi, int lo) {
    const uint64_t u = ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
    double d;
    std::memcpy(&d, &u, 8);
    return d;
}
template <typename T, typename U>
inline T atomicAdd(T *p, U v) {
    return __atomic_fetch_add(p, v, __ATOMIC_SEQ_CST);
}
inline void __syncthreads() { fsv_cpu_syncthreads(); }
using std::max;
using std::min;
inline int min(int a, int b) { return a < b ? a : b; }
inline int max(int a, int b) { return a > b ? a : b; }

// ---- launches: arguments are converted to the kernel's parameter types when
// the launch is made (as the hardware launch copies them) ----
template <typename... P>
struct fsv_cpu_call {
    void (*k)(P...);
    std::tuple<std::decay_t<P>...> args;
    static void run(void *c) {
        auto *s = (fsv_cpu_call *)c;
        std::apply(s->k, s->args);
    }
    static void del(void *c) { delete (fsv_cpu_call *)c; }
    static void *copy(void *c) { return new fsv_cpu_call(*(fsv_cpu_call *)c); }
};
template <typename... P, typename... A>
hipError_t fsv_cpu_launch_k(void (*k)(P...), const char *name, dim3 g, dim3 b, size_t shm, hipStream_t st,
                            hipEvent_t e0, hipEvent_t e1, A &&...a) {
    auto *c = new fsv_cpu_call<P...>{k, std::tuple<std::decay_t<P>...>(std::forward<A>(a)...)};
    return fsv_cpu_launch((const void *)k, name, g, b, shm, st, e0, e1, &fsv_cpu_call<P...>::run, c,
                          &fsv_cpu_call<P...>::del, &fsv_cpu_call<P...>::copy);
}
#define hipLaunchKernelGGL(K, G, B, SHM, ST, ...) \
    (void)fsv_cpu_launch_k(K, #K, dim3(G), dim3(B), (size_t)(SHM), ST, nullptr, nullptr, ##__VA_ARGS__)
template <typename... P, typename... A>
inline void hipExtLaunchKernelGGL(void (*k)(P...), const dim3 &g, const dim3 &b, uint32_t shm, hipStream_t st,
                                  hipEvent_t e0, hipEvent_t e1, uint32_t, A &&...a) {
    (void)fsv_cpu_launch_k(k, "kernel launched with events", g, b, shm, st, e0, e1, std::forward<A>(a)...);
}
#undef HIP_SYMBOL
#define HIP_SYMBOL(x) fsv_cpu_symbol(&(x), sizeof(x))
