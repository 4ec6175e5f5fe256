// HIP kernels for gfx950 (CDNA4) on the dense 2^n amplitude vector:
// excitation rotations over all active amplitude pairs, the adjoint reverse
// step, LDS-staged runs of low-qubit operators, the gather/scatter between
// the dense vector and the compact sector, the one-particle density matrix,
// fills and ordered reductions.
//
// Every reduction is two-stage and ordered (wavefront shuffle -> LDS ->
// per-block partial -> one ordered pass), so results are bitwise
// reproducible run to run; there are no floating-point atomics.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fsv_device.h"
#include "fsv_internal.h"

namespace fsv {

namespace {

template <typename R> struct C2;
template <> struct C2<double> { using T = double2; };
template <> struct C2<float> { using T = float2; };

// Insert zeros at the nt sorted target positions of the pair counter t.
template <typename Idx>
__device__ __forceinline__ Idx insert_zeros(Idx t, const RotOp &op) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k < op.nt) {
            const uint32_t q = op.q[k];
            const Idx lo = t & ((Idx(1) << q) - 1);
            t = ((t >> q) << (q + 1)) | lo;
        }
    }
    return t;
}

// ---------------------------------------------------------------- fills ----
__global__ void k_fill_zero(uint4 *p, size_t n16) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

__global__ void k_fill_tail(unsigned char *p, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

// dst[i] = src[i] for i < n; src may be host memory (pinned, coherent).
__global__ void k_copy_doubles(const double *__restrict__ src, double *__restrict__ dst, int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) dst[i] = src[i];
}

// One amplitude set to (re, 0); vt selects the storage type.
__global__ void k_set_amp(void *psi, int vt, uint64_t x, double re) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    switch (vt) {
    case V_C128: ((double2 *)psi)[x] = make_double2(re, 0.0); break;
    case V_C64: ((float2 *)psi)[x] = make_float2((float)re, 0.f); break;
    case V_F64: ((double *)psi)[x] = re; break;
    default: ((float *)psi)[x] = (float)re; break;
    }
}

// A list of amplitudes psi[idx[i]] = (val[i], 0) (a multi-determinant start).
__global__ void k_set_list(void *psi, int vt, const int64_t *__restrict__ idx, const double *__restrict__ val,
                           int n) {
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
        const int64_t x = idx[i];
        const double re = val[i];
        switch (vt) {
        case V_C128: ((double2 *)psi)[x] = make_double2(re, 0.0); break;
        case V_C64: ((float2 *)psi)[x] = make_float2((float)re, 0.f); break;
        case V_F64: ((double *)psi)[x] = re; break;
        default: ((float *)psi)[x] = (float)re; break;
        }
    }
}

// ------------------------------------------------------------ rotations ----
// psi'_src = c psi_src - s sg psi_dst ; psi'_dst = c psi_dst + s sg psi_src
template <typename R, typename Idx, int PPT>
__global__ __launch_bounds__(1024) void k_rot(typename C2<R>::T *__restrict__ psi, RotOp op,
                                              const double *__restrict__ cs, int k, Idx npairs) {
    using V = typename C2<R>::T;
    const R c = (R)cs[2 * k];
    const R s = (R)cs[2 * k + 1];
    const Idx nthr = (Idx)gridDim.x * blockDim.x;
    for (Idx t0 = (Idx)blockIdx.x * blockDim.x + threadIdx.x; t0 < npairs; t0 += nthr * PPT) {
        V a[PPT], b[PPT];
        Idx xs[PPT], xd[PPT];
        R sg[PPT];
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const Idx t = t0 + (Idx)j * nthr;
            if (t < npairs) {
                const Idx base = insert_zeros<Idx>(t, op);
                xs[j] = base | (Idx)op.src;
                xd[j] = base | (Idx)op.dst;
                const int odd = popc((uint64_t)base & op.par) & 1;
                sg[j] = (odd ? -s : s) * (R)op.sign0;
                a[j] = psi[xs[j]];
                b[j] = psi[xd[j]];
            }
        }
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const Idx t = t0 + (Idx)j * nthr;
            if (t < npairs) {
                V na, nb;
                na.x = c * a[j].x - sg[j] * b[j].x;
                na.y = c * a[j].y - sg[j] * b[j].y;
                nb.x = c * b[j].x + sg[j] * a[j].x;
                nb.y = c * b[j].y + sg[j] * a[j].y;
                psi[xs[j]] = na;
                psi[xd[j]] = nb;
            }
        }
    }
}

// Adjoint step for operator k: partial of Re<lam|T|psi> (T = tau - tau^+),
// then psi <- U^+ psi, lam <- U^+ lam on the same pairs.
template <typename R, typename Idx, int PPT>
__global__ __launch_bounds__(1024) void k_adj(typename C2<R>::T *__restrict__ psi,
                                              typename C2<R>::T *__restrict__ lam, RotOp op,
                                              const double *__restrict__ cs, int k, Idx npairs,
                                              double *__restrict__ partial) {
    using V = typename C2<R>::T;
    const R c = (R)cs[2 * k];
    const R s = (R)cs[2 * k + 1];
    const Idx nthr = (Idx)gridDim.x * blockDim.x;
    double acc = 0.0;
    for (Idx t0 = (Idx)blockIdx.x * blockDim.x + threadIdx.x; t0 < npairs; t0 += nthr * PPT) {
        V pa[PPT], pb[PPT], la[PPT], lb[PPT];
        Idx xs[PPT], xd[PPT];
        int odd[PPT];
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const Idx t = t0 + (Idx)j * nthr;
            if (t < npairs) {
                const Idx base = insert_zeros<Idx>(t, op);
                xs[j] = base | (Idx)op.src;
                xd[j] = base | (Idx)op.dst;
                odd[j] = (popc((uint64_t)base & op.par) & 1) ^ (op.sign0 < 0 ? 1 : 0);
                pa[j] = psi[xs[j]];
                pb[j] = psi[xd[j]];
                la[j] = lam[xs[j]];
                lb[j] = lam[xd[j]];
            }
        }
#pragma unroll
        for (int j = 0; j < PPT; ++j) {
            const Idx t = t0 + (Idx)j * nthr;
            if (t < npairs) {
                // <lam|T psi> on the pair: conj(lam_d) sg psi_s - conj(lam_s) sg psi_d
                double o = (double)lb[j].x * pa[j].x + (double)lb[j].y * pa[j].y -
                           (double)la[j].x * pb[j].x - (double)la[j].y * pb[j].y;
                acc += odd[j] ? -o : o;
                const R sg = odd[j] ? -s : s;
                V na, nb;
                na.x = c * pa[j].x + sg * pb[j].x;
                na.y = c * pa[j].y + sg * pb[j].y;
                nb.x = c * pb[j].x - sg * pa[j].x;
                nb.y = c * pb[j].y - sg * pa[j].y;
                psi[xs[j]] = na;
                psi[xd[j]] = nb;
                na.x = c * la[j].x + sg * lb[j].x;
                na.y = c * la[j].y + sg * lb[j].y;
                nb.x = c * lb[j].x - sg * la[j].x;
                nb.y = c * lb[j].y - sg * la[j].y;
                lam[xs[j]] = na;
                lam[xd[j]] = nb;
            }
        }
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// ------------------------------------------------ LDS-staged fused run ----
// One workgroup per 2^TB-amplitude tile (grid-stride over tiles).  All
// operators of the run have targets below TB, so every pair lies inside one
// tile; the bits above TB only enter the JW sign through the parity mask.
template <typename R, int TB>
__global__ __launch_bounds__(512) void k_rot_fused(typename C2<R>::T *__restrict__ psi,
                                                   const RotOp *__restrict__ ops,
                                                   const double *__restrict__ cs, int k0, int k1,
                                                   uint64_t ntiles) {
    using V = typename C2<R>::T;
    __shared__ V tile[1 << TB];
    for (uint64_t tix = blockIdx.x; tix < ntiles; tix += gridDim.x) {
        const uint64_t hi = tix << TB;
        V *g = psi + hi;
        for (uint32_t i = threadIdx.x; i < (1u << TB); i += blockDim.x) tile[i] = g[i];
        __syncthreads();
        for (int k = k0; k < k1; ++k) {
            const RotOp op = ops[k];
            const R c = (R)cs[2 * k];
            const R s0 = (R)cs[2 * k + 1] * (R)op.sign0 * ((popc(hi & op.par) & 1) ? (R)-1 : (R)1);
            const uint32_t np = 1u << (TB - op.nt);
            for (uint32_t t = threadIdx.x; t < np; t += blockDim.x) {
                const uint32_t base = insert_zeros<uint32_t>(t, op);
                const uint32_t xs = base | (uint32_t)op.src, xd = base | (uint32_t)op.dst;
                const R sg = (popc((uint32_t)(base & (uint32_t)op.par)) & 1) ? -s0 : s0;
                const V a = tile[xs], b = tile[xd];
                V na, nb;
                na.x = c * a.x - sg * b.x;
                na.y = c * a.y - sg * b.y;
                nb.x = c * b.x + sg * a.x;
                nb.y = c * b.y + sg * a.y;
                tile[xs] = na;
                tile[xd] = nb;
            }
            __syncthreads();
        }
        for (uint32_t i = threadIdx.x; i < (1u << TB); i += blockDim.x) g[i] = tile[i];
        __syncthreads();
    }
}

// Adjoint of an LDS-staged fused run: the tile's psi and lam are staged, the
// run's operators are undone last to first, and each operator's share of
// Re<lam|T|psi> (T = tau - tau^+, taken before the operator is undone) is
// summed over the workgroup's tiles and written to
// partial[k * pstride + blockIdx.x].  The sign of a pair is that of k_adj:
// sign0 times the parity of the pair's index, split into the tile bits and
// the bits above.
constexpr int kMaxFusedRun = 64;

template <typename R, int TB>
__global__ __launch_bounds__(512) void k_adj_fused(typename C2<R>::T *__restrict__ psi,
                                                   typename C2<R>::T *__restrict__ lam,
                                                   const RotOp *__restrict__ ops,
                                                   const double *__restrict__ cs, int k0, int k1,
                                                   uint64_t ntiles, double *__restrict__ partial, int pstride) {
    using V = typename C2<R>::T;
    extern __shared__ double smem[];
    V *tp = (V *)smem;          // psi tile
    V *tl = tp + (1 << TB);     // lam tile
    __shared__ double part[kMaxFusedRun];
    const int nops = k1 - k0;
    for (int i = threadIdx.x; i < nops; i += blockDim.x) part[i] = 0.0;
    for (uint64_t tix = blockIdx.x; tix < ntiles; tix += gridDim.x) {
        const uint64_t hi = tix << TB;
        V *gp = psi + hi, *gl = lam + hi;
        for (uint32_t i = threadIdx.x; i < (1u << TB); i += blockDim.x) {
            tp[i] = gp[i];
            tl[i] = gl[i];
        }
        __syncthreads();
        for (int k = k1 - 1; k >= k0; --k) {
            const RotOp op = ops[k];
            const R c = (R)cs[2 * k];
            const bool flip0 = (op.sign0 < 0) != ((popc(hi & op.par) & 1) != 0);
            const uint32_t np = 1u << (TB - op.nt);
            double acc = 0.0;
            for (uint32_t t = threadIdx.x; t < np; t += blockDim.x) {
                const uint32_t base = insert_zeros<uint32_t>(t, op);
                const uint32_t xs = base | (uint32_t)op.src, xd = base | (uint32_t)op.dst;
                const bool odd = flip0 != ((popc((uint32_t)(base & (uint32_t)op.par)) & 1) != 0);
                const V pa = tp[xs], pb = tp[xd], la = tl[xs], lb = tl[xd];
                const double o = (double)lb.x * pa.x + (double)lb.y * pa.y - (double)la.x * pb.x -
                                 (double)la.y * pb.y;
                acc += odd ? -o : o;
                const R sg = odd ? -(R)cs[2 * k + 1] : (R)cs[2 * k + 1];
                V na, nb;
                na.x = c * pa.x + sg * pb.x;
                na.y = c * pa.y + sg * pb.y;
                nb.x = c * pb.x - sg * pa.x;
                nb.y = c * pb.y - sg * pa.y;
                tp[xs] = na;
                tp[xd] = nb;
                na.x = c * la.x + sg * lb.x;
                na.y = c * la.y + sg * lb.y;
                nb.x = c * lb.x - sg * la.x;
                nb.y = c * lb.y - sg * la.y;
                tl[xs] = na;
                tl[xd] = nb;
            }
            // the workgroup sum also orders this operator's LDS updates before the next
            const double tot = block_sum(acc);
            if (threadIdx.x == 0) part[k - k0] += tot;
        }
        for (uint32_t i = threadIdx.x; i < (1u << TB); i += blockDim.x) {
            gp[i] = tp[i];
            gl[i] = tl[i];
        }
        __syncthreads();
    }
    for (int i = threadIdx.x; i < nops; i += blockDim.x) partial[(size_t)(k0 + i) * pstride + blockIdx.x] = part[i];
}

// Energy and gradients in one launch: out[0] = sum_{b < ecount[0]} epart[b],
// out[1 + k] = 2 sum_{b < gcount[k]} gpart[k * stride + b]; each row summed
// exactly as k_reduce_rows sums it.
__global__ void k_reduce_eg(const double *__restrict__ epart, const int *__restrict__ ecount,
                            const double *__restrict__ gpart, const int *__restrict__ gcount, int stride,
                            double *__restrict__ out) {
    const int r = blockIdx.x;
    const double *partial = r == 0 ? epart : gpart + (size_t)(r - 1) * stride;
    const int n = r == 0 ? ecount[0] : gcount[r - 1];
    double acc = 0.0;
    for (int b = threadIdx.x; b < n; b += blockDim.x) acc += partial[b];
    acc = block_sum(acc);
    if (threadIdx.x == 0) out[r] = r == 0 ? acc : 2.0 * acc;
}

// Row-wise ordered reduction: out[r] = scale * sum_{b < counts[r]} partial[r*stride + b].
__global__ void k_reduce_rows(const double *__restrict__ partial, const int *__restrict__ counts,
                              int stride, double scale, double *__restrict__ out) {
    const int r = blockIdx.x;
    const int n = counts[r];
    double acc = 0.0;
    for (int b = threadIdx.x; b < n; b += blockDim.x) acc += partial[(size_t)r * stride + b];
    acc = block_sum(acc);
    if (threadIdx.x == 0) out[r] = scale * acc;
}

// ------------------------------------------------- sector gather/scatter ----
// Dense amplitude of (Ia, Ib) -> alpha-first compact value.  The sign converts
// the qubit-ordered creator product into the alpha-string-first product.
template <typename R>
__global__ void k_gather(const typename C2<R>::T *__restrict__ psi, const uint64_t *__restrict__ Xa,
                         const uint64_t *__restrict__ Xb, const uint32_t *__restrict__ sa,
                         const uint32_t *__restrict__ PPb, int64_t nsb, double2 *__restrict__ C) {
    const int64_t Ia = blockIdx.y;
    for (int64_t Ib = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; Ib < nsb;
         Ib += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t x = Xa[Ia] | Xb[Ib];
        const bool neg = popc(sa[Ia] & PPb[Ib]) & 1;
        const typename C2<R>::T v = psi[x];
        double2 o;
        o.x = neg ? -(double)v.x : (double)v.x;
        o.y = neg ? -(double)v.y : (double)v.y;
        C[Ia * nsb + Ib] = o;
    }
}

template <typename R>
__global__ void k_scatter(typename C2<R>::T *__restrict__ lam, const double2 *__restrict__ S,
                          const uint64_t *__restrict__ Xa, const uint64_t *__restrict__ Xb,
                          const uint32_t *__restrict__ sa, const uint32_t *__restrict__ PPb,
                          int64_t nsb) {
    const int64_t Ia = blockIdx.y;
    for (int64_t Ib = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; Ib < nsb;
         Ib += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t x = Xa[Ia] | Xb[Ib];
        const bool neg = popc(sa[Ia] & PPb[Ib]) & 1;
        const double2 v = S[Ia * nsb + Ib];
        typename C2<R>::T o;
        o.x = (R)(neg ? -v.x : v.x);
        o.y = (R)(neg ? -v.y : v.y);
        lam[x] = o;
    }
}

// ------------------------------------------------------------- 1-RDM ----
// O[I*nexc + e] = s_e * sum_c conj(A[I][c]) A[J_e][c]; one wavefront per (I, e).
__global__ __launch_bounds__(256) void k_rdm_overlap(const double2 *__restrict__ A, int64_t ncols,
                                                     const uint32_t *__restrict__ exc, int nexc,
                                                     double2 *__restrict__ O) {
    const int64_t I = blockIdx.x;
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    const int nw = blockDim.x / kWave;
    for (int e = wid; e < nexc; e += nw) {
        const uint32_t w = exc[I * nexc + e];
        const int64_t J = w & 0xFFFFu;
        double re = 0.0, im = 0.0;
        for (int64_t c = lane; c < ncols; c += kWave) {
            const double2 a = A[I * ncols + c], b = A[J * ncols + c];
            re += a.x * b.x + a.y * b.y;
            im += a.x * b.y - a.y * b.x;
        }
        re = wave_sum(re);
        im = wave_sum(im);
        if (lane == 0) {
            const bool neg = w >> 31;
            O[I * nexc + e] = make_double2(neg ? -re : re, neg ? -im : im);
        }
    }
}

__global__ void k_rdm_bin(const double2 *__restrict__ O, const int32_t *__restrict__ off,
                          const int32_t *__restrict__ idx, double2 *__restrict__ out) {
    const int b = blockIdx.x;
    double re = 0.0, im = 0.0;
    for (int k = off[b] + threadIdx.x; k < off[b + 1]; k += blockDim.x) {
        const double2 v = O[idx[k]];
        re += v.x;
        im += v.y;
    }
    re = block_sum(re);
    im = block_sum(im);
    if (threadIdx.x == 0) out[b] = make_double2(re, im);
}

template <typename R, typename Idx>
hipError_t rot_dispatch(void *psi, const RotOp &op, const double *cs, int k, uint64_t npairs,
                        Shape sh, hipStream_t st) {
    using V = typename C2<R>::T;
    const unsigned grid = rot_grid(npairs, sh);
    switch (sh.ppt) {
    case 1: hipLaunchKernelGGL((k_rot<R, Idx, 1>), dim3(grid), dim3(sh.block), 0, st, (V *)psi, op, cs, k, (Idx)npairs); break;
    case 2: hipLaunchKernelGGL((k_rot<R, Idx, 2>), dim3(grid), dim3(sh.block), 0, st, (V *)psi, op, cs, k, (Idx)npairs); break;
    case 8: hipLaunchKernelGGL((k_rot<R, Idx, 8>), dim3(grid), dim3(sh.block), 0, st, (V *)psi, op, cs, k, (Idx)npairs); break;
    default: hipLaunchKernelGGL((k_rot<R, Idx, 4>), dim3(grid), dim3(sh.block), 0, st, (V *)psi, op, cs, k, (Idx)npairs); break;
    }
    return hipGetLastError();
}

template <typename R, typename Idx>
hipError_t adj_dispatch(void *psi, void *lam, const RotOp &op, const double *cs, int k,
                        uint64_t npairs, Shape sh, double *partial, hipStream_t st) {
    using V = typename C2<R>::T;
    const unsigned grid = rot_grid(npairs, sh);
    switch (sh.ppt) {
    case 1: hipLaunchKernelGGL((k_adj<R, Idx, 1>), dim3(grid), dim3(sh.block), 0, st, (V *)psi, (V *)lam, op, cs, k, (Idx)npairs, partial); break;
    case 2: hipLaunchKernelGGL((k_adj<R, Idx, 2>), dim3(grid), dim3(sh.block), 0, st, (V *)psi, (V *)lam, op, cs, k, (Idx)npairs, partial); break;
    case 8: hipLaunchKernelGGL((k_adj<R, Idx, 8>), dim3(grid), dim3(sh.block), 0, st, (V *)psi, (V *)lam, op, cs, k, (Idx)npairs, partial); break;
    default: hipLaunchKernelGGL((k_adj<R, Idx, 4>), dim3(grid), dim3(sh.block), 0, st, (V *)psi, (V *)lam, op, cs, k, (Idx)npairs, partial); break;
    }
    return hipGetLastError();
}

}  // namespace

int max_grid() { return kMaxGrid; }

void init_kernels() {
    init_sigma_kernels();
    init_fused_kernels();
    // the adjoint fused run stages psi and lam tiles: 128 KiB of dynamic LDS
    (void)hipFuncSetAttribute((const void *)k_adj_fused<double, 12>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              2 * (1 << 12) * (int)sizeof(double2));
    (void)hipFuncSetAttribute((const void *)k_adj_fused<float, 13>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              2 * (1 << 13) * (int)sizeof(float2));
    (void)hipGetLastError();
}

int max_fused_run() { return kMaxFusedRun; }

unsigned fused_grid(uint64_t n_amps, int tile_bits) {
    const uint64_t ntiles = n_amps >> tile_bits;
    return (unsigned)(ntiles < (uint64_t)kMaxGrid ? ntiles : (uint64_t)kMaxGrid);
}

unsigned rot_grid(uint64_t npairs, Shape sh) {
    const uint64_t per = (uint64_t)sh.block * (uint64_t)sh.ppt;
    uint64_t g = (npairs + per - 1) / per;
    if (g < 1) g = 1;
    if (g > (uint64_t)kMaxGrid) g = kMaxGrid;
    return (unsigned)g;
}

hipError_t launch_fill_zero(void *ptr, size_t bytes, hipStream_t st) {
    const size_t n16 = bytes / 16;
    if (n16) {
        const int block = 256;
        size_t grid = (n16 + block - 1) / block;
        if (grid > 65536) grid = 65536;
        hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)grid), dim3(block), 0, st, (uint4 *)ptr, n16);
    }
    const size_t tail = bytes - n16 * 16;
    if (tail) {
        hipLaunchKernelGGL(k_fill_tail, dim3(1), dim3(64), 0, st, (unsigned char *)ptr + n16 * 16, tail);
    }
    return hipGetLastError();
}

hipError_t launch_copy_doubles(const double *src, double *dst, int n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_doubles, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_set_amp(void *psi, int vt, uint64_t x, double re, hipStream_t st) {
    hipLaunchKernelGGL(k_set_amp, dim3(1), dim3(64), 0, st, psi, vt, x, re);
    return hipGetLastError();
}

hipError_t launch_set_list(void *psi, int vt, const int64_t *idx, const double *val, int n, hipStream_t st) {
    hipLaunchKernelGGL(k_set_list, dim3(blocks_for(n, 256)), dim3(256), 0, st, psi, vt, idx, val, n);
    return hipGetLastError();
}

hipError_t launch_rot(int precision, bool wide, void *psi, const RotOp &op, const double *cs,
                      int k, uint64_t npairs, Shape sh, hipStream_t st) {
    if (precision == 0)
        return wide ? rot_dispatch<double, uint64_t>(psi, op, cs, k, npairs, sh, st)
                    : rot_dispatch<double, uint32_t>(psi, op, cs, k, npairs, sh, st);
    return wide ? rot_dispatch<float, uint64_t>(psi, op, cs, k, npairs, sh, st)
                : rot_dispatch<float, uint32_t>(psi, op, cs, k, npairs, sh, st);
}

hipError_t launch_adj(int precision, bool wide, void *psi, void *lam, const RotOp &op,
                      const double *cs, int k, uint64_t npairs, Shape sh, double *partial,
                      hipStream_t st) {
    if (precision == 0)
        return wide ? adj_dispatch<double, uint64_t>(psi, lam, op, cs, k, npairs, sh, partial, st)
                    : adj_dispatch<double, uint32_t>(psi, lam, op, cs, k, npairs, sh, partial, st);
    return wide ? adj_dispatch<float, uint64_t>(psi, lam, op, cs, k, npairs, sh, partial, st)
                : adj_dispatch<float, uint32_t>(psi, lam, op, cs, k, npairs, sh, partial, st);
}

hipError_t launch_rot_fused(int precision, void *psi, const RotOp *ops_dev, const double *cs,
                            int k0, int k1, int tile_bits, uint64_t n_amps, hipStream_t st) {
    const uint64_t ntiles = n_amps >> tile_bits;
    const unsigned grid = fused_grid(n_amps, tile_bits);
    if (precision == 0) {
        if (tile_bits != 12) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_rot_fused<double, 12>), dim3(grid), dim3(512), 0, st, (double2 *)psi,
                           ops_dev, cs, k0, k1, ntiles);
    } else {
        if (tile_bits != 13) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_rot_fused<float, 13>), dim3(grid), dim3(512), 0, st, (float2 *)psi,
                           ops_dev, cs, k0, k1, ntiles);
    }
    return hipGetLastError();
}

hipError_t launch_adj_fused(int precision, void *psi, void *lam, const RotOp *ops_dev, const double *cs,
                            int k0, int k1, int tile_bits, uint64_t n_amps, double *partial, int pstride,
                            hipStream_t st) {
    if (k1 - k0 < 1 || k1 - k0 > kMaxFusedRun) return hipErrorInvalidValue;
    const uint64_t ntiles = n_amps >> tile_bits;
    const unsigned grid = fused_grid(n_amps, tile_bits);
    if (precision == 0) {
        if (tile_bits != 12) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_adj_fused<double, 12>), dim3(grid), dim3(512), 2 * (1 << 12) * sizeof(double2), st,
                           (double2 *)psi, (double2 *)lam, ops_dev, cs, k0, k1, ntiles, partial, pstride);
    } else {
        if (tile_bits != 13) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_adj_fused<float, 13>), dim3(grid), dim3(512), 2 * (1 << 13) * sizeof(float2), st,
                           (float2 *)psi, (float2 *)lam, ops_dev, cs, k0, k1, ntiles, partial, pstride);
    }
    return hipGetLastError();
}

hipError_t launch_reduce_eg(const double *epart, const int *ecount, const double *gpart, const int *gcount,
                            int stride, int k, double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_reduce_eg, dim3((unsigned)(k + 1)), dim3(256), 0, st, epart, ecount, gpart, gcount, stride,
                       out);
    return hipGetLastError();
}

hipError_t launch_reduce_rows(const double *partial, const int *counts, int stride, int rows,
                              double scale, double *out, hipStream_t st) {
    if (rows <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_reduce_rows, dim3(rows), dim3(256), 0, st, partial, counts, stride, scale, out);
    return hipGetLastError();
}

hipError_t launch_gather(int precision, const void *psi, const uint64_t *Xa, const uint64_t *Xb,
                         const uint32_t *sa, const uint32_t *PPb, int64_t nsa, int64_t nsb,
                         double2 *C, hipStream_t st) {
    const dim3 grid(blocks_for(nsb, 256) > 64 ? 64 : blocks_for(nsb, 256), (unsigned)nsa);
    if (precision == 0)
        hipLaunchKernelGGL(k_gather<double>, grid, dim3(256), 0, st, (const double2 *)psi, Xa, Xb, sa, PPb, nsb, C);
    else
        hipLaunchKernelGGL(k_gather<float>, grid, dim3(256), 0, st, (const float2 *)psi, Xa, Xb, sa, PPb, nsb, C);
    return hipGetLastError();
}

hipError_t launch_scatter(int precision, void *lam, const double2 *S, const uint64_t *Xa,
                          const uint64_t *Xb, const uint32_t *sa, const uint32_t *PPb,
                          int64_t nsa, int64_t nsb, hipStream_t st) {
    const dim3 grid(blocks_for(nsb, 256) > 64 ? 64 : blocks_for(nsb, 256), (unsigned)nsa);
    if (precision == 0)
        hipLaunchKernelGGL(k_scatter<double>, grid, dim3(256), 0, st, (double2 *)lam, S, Xa, Xb, sa, PPb, nsb);
    else
        hipLaunchKernelGGL(k_scatter<float>, grid, dim3(256), 0, st, (float2 *)lam, S, Xa, Xb, sa, PPb, nsb);
    return hipGetLastError();
}

hipError_t launch_rdm_overlap(const double2 *A, int64_t nrows, int64_t ncols,
                              const uint32_t *exc, int nexc, double2 *O, hipStream_t st) {
    hipLaunchKernelGGL(k_rdm_overlap, dim3((unsigned)nrows), dim3(256), 0, st, A, ncols, exc, nexc, O);
    return hipGetLastError();
}

hipError_t launch_rdm_bin(const double2 *O, const int32_t *off, const int32_t *idx, int nbins,
                          double2 *out, hipStream_t st) {
    hipLaunchKernelGGL(k_rdm_bin, dim3(nbins), dim3(256), 0, st, O, off, idx, out);
    return hipGetLastError();
}

}  // namespace fsv
