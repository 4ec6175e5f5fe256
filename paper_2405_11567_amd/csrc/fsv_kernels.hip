// HIP kernels for gfx950 (CDNA4): excitation rotations on the dense 2^n
// amplitude vector, the adjoint reverse step, sector gather/scatter, the
// sector Hamiltonian product and the one-particle density matrix.
//
// Every reduction is two-stage and ordered (wavefront shuffle -> LDS ->
// per-block partial -> one ordered pass), so results are bitwise
// reproducible run to run; there are no floating-point atomics.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fsv_internal.h"

namespace fsv {

namespace {

constexpr int kMaxGrid = 8192;
constexpr int kWave = 64;

template <typename R> struct C2;
template <> struct C2<double> { using T = double2; };
template <> struct C2<float> { using T = float2; };

__device__ __forceinline__ int popc(uint64_t v) { return __popcll(v); }
__device__ __forceinline__ int popc(uint32_t v) { return __popc(v); }

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

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Block-wide ordered sum; every thread gets the result.  blockDim <= 1024.
__device__ double block_sum(double v) {
    __shared__ double red[1024 / kWave];
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    const int nw = (blockDim.x + kWave - 1) / kWave;
    v = wave_sum(v);
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w];  // same order in every thread
    __syncthreads();
    return s;
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

template <typename R>
__global__ void k_set_amp(typename C2<R>::T *psi, uint64_t x, double re) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        typename C2<R>::T v;
        v.x = (R)re;
        v.y = (R)0;
        psi[x] = v;
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
// One workgroup per 2^tb-amplitude tile (grid-stride over tiles).  All
// operators of the run have targets below tb, so every pair lies inside one
// tile; the bits above tb only enter the JW sign through the parity mask.
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
                         const uint32_t *__restrict__ PPb, int64_t nsa, int64_t nsb,
                         double2 *__restrict__ C) {
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
                          int64_t nsa, int64_t nsb) {
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

// ------------------------------------------------------- sector sigma ----
// out[I][:] = sum_k val[k] * in[col[k]][:]   (one block per output row)
__global__ void k_spmm_rows(const int64_t *__restrict__ rowptr, const int32_t *__restrict__ col,
                            const double *__restrict__ val, const double2 *__restrict__ in,
                            double2 *__restrict__ out, int64_t ncols) {
    const int64_t I = blockIdx.y;
    const int64_t k0 = rowptr[I], k1 = rowptr[I + 1];
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < ncols;
         c += (int64_t)gridDim.x * blockDim.x) {
        double ar = 0.0, ai = 0.0;
        for (int64_t k = k0; k < k1; ++k) {
            const double v = val[k];
            const double2 x = in[(int64_t)col[k] * ncols + c];
            ar += v * x.x;
            ai += v * x.y;
        }
        out[I * ncols + c] = make_double2(ar, ai);
    }
}

// Alpha-beta two-body term: S[Ia][Ib] += sum_{e in exc(Ia)} sum_{f in exc(Ib)}
// s_e s_f (pq_e|rs_f) C[J_e][J_f].
constexpr int kMaxExc = 96;
__global__ __launch_bounds__(256) void k_sigma_ab(const uint32_t *__restrict__ excA, int nexcA,
                                                  const uint32_t *__restrict__ excB, int nexcB,
                                                  const double *__restrict__ g, int M,
                                                  const double2 *__restrict__ C,
                                                  double2 *__restrict__ S, int64_t nsb) {
    __shared__ uint32_t ea[kMaxExc];
    const int64_t Ia = blockIdx.x;
    for (int e = threadIdx.x; e < nexcA; e += blockDim.x) ea[e] = excA[Ia * nexcA + e];
    __syncthreads();
    const int M2 = M * M;
    for (int64_t Ib = threadIdx.x; Ib < nsb; Ib += blockDim.x) {
        double ar = 0.0, ai = 0.0;
        for (int f = 0; f < nexcB; ++f) {
            const uint32_t eb = excB[Ib * nexcB + f];
            const int64_t Jb = eb & 0xFFFFu;
            const int rs = (eb >> 16) & 0x1FFu;
            const bool nb = eb >> 31;
            double br = 0.0, bi = 0.0;
            for (int e = 0; e < nexcA; ++e) {
                const uint32_t w = ea[e];
                const int64_t Ja = w & 0xFFFFu;
                const int pq = (w >> 16) & 0x1FFu;
                const double gv = g[pq * M2 + rs];
                const double2 x = C[Ja * nsb + Jb];
                const double sgv = (w >> 31) ? -gv : gv;
                br += sgv * x.x;
                bi += sgv * x.y;
            }
            ar += nb ? -br : br;
            ai += nb ? -bi : bi;
        }
        double2 o = S[Ia * nsb + Ib];
        o.x += ar;
        o.y += ai;
        S[Ia * nsb + Ib] = o;
    }
}

// Same term with the source rows staged in LDS: for output row Ia the
// alpha excitations are taken ec at a time; their rows C[J_e][:] and the
// weights W[e][rs] = s_e (pq_e|rs) sit in LDS, and each thread gathers its
// beta excitations from there.
__global__ __launch_bounds__(512) void k_sigma_ab_lds(const uint32_t *__restrict__ excA, int nexcA,
                                                      const uint32_t *__restrict__ excB, int nexcB,
                                                      const double *__restrict__ g, int M,
                                                      const double2 *__restrict__ C,
                                                      double2 *__restrict__ S, int64_t nsb, int ec) {
    extern __shared__ double2 smem[];
    double2 *rows = smem;                                // ec * nsb
    double *W = (double *)(smem + (int64_t)ec * nsb);    // ec * M2
    const int64_t Ia = blockIdx.x;
    const int M2 = M * M;
    for (int e0 = 0; e0 < nexcA; e0 += ec) {
        const int ne = min(ec, nexcA - e0);
        for (int e = 0; e < ne; ++e) {
            const uint32_t w = excA[Ia * nexcA + e0 + e];
            const int64_t Ja = w & 0xFFFFu;
            const int pq = (w >> 16) & 0x1FFu;
            const double sa = (w >> 31) ? -1.0 : 1.0;
            for (int64_t c = threadIdx.x; c < nsb; c += blockDim.x) rows[e * nsb + c] = C[Ja * nsb + c];
            for (int rs = threadIdx.x; rs < M2; rs += blockDim.x) W[e * M2 + rs] = sa * g[pq * M2 + rs];
        }
        __syncthreads();
        for (int64_t Ib = threadIdx.x; Ib < nsb; Ib += blockDim.x) {
            double ar = 0.0, ai = 0.0;
            for (int f = 0; f < nexcB; ++f) {
                const uint32_t eb = excB[Ib * nexcB + f];
                const int64_t Jb = eb & 0xFFFFu;
                const int rs = (eb >> 16) & 0x1FFu;
                double br = 0.0, bi = 0.0;
                for (int e = 0; e < ne; ++e) {
                    const double wv = W[e * M2 + rs];
                    const double2 x = rows[e * nsb + Jb];
                    br += wv * x.x;
                    bi += wv * x.y;
                }
                if (eb >> 31) {
                    ar -= br;
                    ai -= bi;
                } else {
                    ar += br;
                    ai += bi;
                }
            }
            double2 o = S[Ia * nsb + Ib];
            o.x += ar;
            o.y += ai;
            S[Ia * nsb + Ib] = o;
        }
        __syncthreads();
    }
}

__global__ void k_transpose(const double2 *__restrict__ in, double2 *__restrict__ out,
                            int64_t rows, int64_t cols) {
    __shared__ double2 t[32][33];
    const int64_t c0 = (int64_t)blockIdx.x * 32, r0 = (int64_t)blockIdx.y * 32;
    for (int j = threadIdx.y; j < 32; j += blockDim.y) {
        const int64_t r = r0 + j, c = c0 + threadIdx.x;
        if (r < rows && c < cols) t[j][threadIdx.x] = in[r * cols + c];
    }
    __syncthreads();
    for (int j = threadIdx.y; j < 32; j += blockDim.y) {
        const int64_t c = c0 + j, r = r0 + threadIdx.x;
        if (r < rows && c < cols) out[c * rows + r] = t[threadIdx.x][j];
    }
}

// S[Ia][Ib] += ST[Ib][Ia] + ecore C[Ia][Ib], and per-block partial Re<C|S>.
__global__ void k_combine(double2 *__restrict__ S, const double2 *__restrict__ ST,
                          const double2 *__restrict__ C, double ecore, int64_t nsa, int64_t nsb,
                          double *__restrict__ partial) {
    const int64_t dim = nsa * nsb;
    double acc = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < dim;
         r += (int64_t)gridDim.x * blockDim.x) {
        const int64_t Ia = r / nsb, Ib = r - Ia * nsb;
        const double2 c = C[r];
        const double2 t = ST[Ib * nsa + Ia];
        double2 s = S[r];
        s.x += t.x + ecore * c.x;
        s.y += t.y + ecore * c.y;
        S[r] = s;
        acc += c.x * s.x + c.y * s.y;
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
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

// ------------------------------------------ sector-compressed rotations ----
// Active pair (u, v): alpha pair u of the operator's alpha list (row u when it
// has no alpha part) and beta pair v (column v when it has no beta part).
// Workgroups tile u with blockIdx.y (stride gridDim.y) and v with blockIdx.x
// and the threads.
struct CGrid {
    unsigned gx, gy, block;
};

__host__ __device__ inline CGrid cgrid_of(const PairOp &op, int64_t nsa, int64_t nsb) {
    const int64_t na = op.nA >= 0 ? op.nA : nsa, nb = op.nB >= 0 ? op.nB : nsb;
    CGrid g;
    g.block = nb <= 64 ? 64u : (nb <= 128 ? 128u : 256u);
    const int64_t gy = na < 1024 ? (na > 0 ? na : 1) : 1024;
    int64_t gx = (nb + g.block - 1) / g.block;
    const int64_t cap = kMaxGrid / gy > 0 ? kMaxGrid / gy : 1;
    if (gx > cap) gx = cap;
    if (gx < 1) gx = 1;
    g.gx = (unsigned)gx;
    g.gy = (unsigned)gy;
    return g;
}

__device__ __forceinline__ void cpair_row(const PairOp &op, const uint32_t *__restrict__ lists,
                                          int64_t u, int64_t &ia, int64_t &ia2, bool &neg) {
    if (op.nA >= 0) {
        const uint32_t e = lists[op.offA + u];
        ia = e & 0x7FFFu;
        ia2 = (e >> 15) & 0x7FFFu;
        neg = (op.sign0 < 0) ^ ((e >> 31) != 0);
    } else {
        ia = ia2 = u;
        neg = op.sign0 < 0;
    }
}

__device__ __forceinline__ void cpair_col(const PairOp &op, const uint32_t *__restrict__ lists,
                                          int64_t v, int64_t &ib, int64_t &ib2, bool &neg) {
    if (op.nB >= 0) {
        const uint32_t e = lists[op.offB + v];
        ib = e & 0x7FFFu;
        ib2 = (e >> 15) & 0x7FFFu;
        neg ^= (e >> 31) != 0;
    } else {
        ib = ib2 = v;
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_crot(typename C2<R>::T *__restrict__ psi, PairOp op,
                                              const uint32_t *__restrict__ lists,
                                              const double *__restrict__ cs, int k, int64_t nsa,
                                              int64_t nsb) {
    using V = typename C2<R>::T;
    const R c = (R)cs[2 * k], s = (R)cs[2 * k + 1];
    const int64_t na = op.nA >= 0 ? op.nA : nsa, nb = op.nB >= 0 ? op.nB : nsb;
    for (int64_t u = blockIdx.y; u < na; u += gridDim.y) {
        int64_t ia, ia2;
        bool nrow;
        cpair_row(op, lists, u, ia, ia2, nrow);
        for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nb;
             v += (int64_t)gridDim.x * blockDim.x) {
            int64_t ib, ib2;
            bool neg = nrow;
            cpair_col(op, lists, v, ib, ib2, neg);
            const int64_t xs = ia * nsb + ib, xd = ia2 * nsb + ib2;
            const R sg = neg ? -s : s;
            const V a = psi[xs], b = psi[xd];
            V na_, nb_;
            na_.x = c * a.x - sg * b.x;
            na_.y = c * a.y - sg * b.y;
            nb_.x = c * b.x + sg * a.x;
            nb_.y = c * b.y + sg * a.y;
            psi[xs] = na_;
            psi[xd] = nb_;
        }
    }
}

template <typename R>
__global__ __launch_bounds__(256) void k_cadj(typename C2<R>::T *__restrict__ psi,
                                              typename C2<R>::T *__restrict__ lam, PairOp op,
                                              const uint32_t *__restrict__ lists,
                                              const double *__restrict__ cs, int k, int64_t nsa,
                                              int64_t nsb, double *__restrict__ partial) {
    using V = typename C2<R>::T;
    const R c = (R)cs[2 * k], s = (R)cs[2 * k + 1];
    const int64_t na = op.nA >= 0 ? op.nA : nsa, nb = op.nB >= 0 ? op.nB : nsb;
    double acc = 0.0;
    for (int64_t u = blockIdx.y; u < na; u += gridDim.y) {
        int64_t ia, ia2;
        bool nrow;
        cpair_row(op, lists, u, ia, ia2, nrow);
        for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nb;
             v += (int64_t)gridDim.x * blockDim.x) {
            int64_t ib, ib2;
            bool neg = nrow;
            cpair_col(op, lists, v, ib, ib2, neg);
            const int64_t xs = ia * nsb + ib, xd = ia2 * nsb + ib2;
            const V a = psi[xs], b = psi[xd], la = lam[xs], lb = lam[xd];
            const double o = (double)lb.x * a.x + (double)lb.y * a.y - (double)la.x * b.x -
                             (double)la.y * b.y;
            acc += neg ? -o : o;
            const R sg = neg ? -s : s;
            V t0, t1;
            t0.x = c * a.x + sg * b.x;
            t0.y = c * a.y + sg * b.y;
            t1.x = c * b.x - sg * a.x;
            t1.y = c * b.y - sg * a.y;
            psi[xs] = t0;
            psi[xd] = t1;
            t0.x = c * la.x + sg * lb.x;
            t0.y = c * la.y + sg * lb.y;
            t1.x = c * lb.x - sg * la.x;
            t1.y = c * lb.y - sg * la.y;
            lam[xs] = t0;
            lam[xd] = t1;
        }
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = acc;
}

__global__ void k_cvt_f2d(const float2 *__restrict__ in, double2 *__restrict__ out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = make_double2((double)in[i].x, (double)in[i].y);
}

__global__ void k_cvt_d2f(const double2 *__restrict__ in, float2 *__restrict__ out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = make_float2((float)in[i].x, (float)in[i].y);
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

unsigned blocks_for(int64_t n, int block) {
    int64_t b = (n + block - 1) / block;
    if (b < 1) b = 1;
    if (b > kMaxGrid) b = kMaxGrid;
    return (unsigned)b;
}

}  // namespace

int max_grid() { return kMaxGrid; }

// LDS budget of the staged sigma kernel: up to the 160 KiB of a gfx950 CU when
// the runtime grants it (set once, outside any stream capture).
static int g_lds_max = -1;

void init_kernels() {
    if (g_lds_max > 0) return;
    g_lds_max = 65536;
    if (hipFuncSetAttribute((const void *)k_sigma_ab_lds, hipFuncAttributeMaxDynamicSharedMemorySize,
                            163840) == hipSuccess)
        g_lds_max = 163840;
    (void)hipGetLastError();
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

hipError_t launch_set_amp(void *psi, int precision, uint64_t x, double re, hipStream_t st) {
    if (precision == 0)
        hipLaunchKernelGGL(k_set_amp<double>, dim3(1), dim3(64), 0, st, (double2 *)psi, x, re);
    else
        hipLaunchKernelGGL(k_set_amp<float>, dim3(1), dim3(64), 0, st, (float2 *)psi, x, re);
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
    const unsigned grid = (unsigned)(ntiles < (uint64_t)kMaxGrid ? ntiles : (uint64_t)kMaxGrid);
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
        hipLaunchKernelGGL(k_gather<double>, grid, dim3(256), 0, st, (const double2 *)psi, Xa, Xb, sa, PPb, nsa, nsb, C);
    else
        hipLaunchKernelGGL(k_gather<float>, grid, dim3(256), 0, st, (const float2 *)psi, Xa, Xb, sa, PPb, nsa, nsb, C);
    return hipGetLastError();
}

hipError_t launch_scatter(int precision, void *lam, const double2 *S, const uint64_t *Xa,
                          const uint64_t *Xb, const uint32_t *sa, const uint32_t *PPb,
                          int64_t nsa, int64_t nsb, hipStream_t st) {
    const dim3 grid(blocks_for(nsb, 256) > 64 ? 64 : blocks_for(nsb, 256), (unsigned)nsa);
    if (precision == 0)
        hipLaunchKernelGGL(k_scatter<double>, grid, dim3(256), 0, st, (double2 *)lam, S, Xa, Xb, sa, PPb, nsa, nsb);
    else
        hipLaunchKernelGGL(k_scatter<float>, grid, dim3(256), 0, st, (float2 *)lam, S, Xa, Xb, sa, PPb, nsa, nsb);
    return hipGetLastError();
}

hipError_t launch_spmm_rows(const int64_t *rowptr, const int32_t *col, const double *val,
                            const double2 *in, double2 *out, int64_t nrows, int64_t ncols,
                            hipStream_t st) {
    const dim3 grid(blocks_for(ncols, 256) > 64 ? 64 : blocks_for(ncols, 256), (unsigned)nrows);
    hipLaunchKernelGGL(k_spmm_rows, grid, dim3(256), 0, st, rowptr, col, val, in, out, ncols);
    return hipGetLastError();
}

hipError_t launch_sigma_ab(const uint32_t *excA, int nexcA, const uint32_t *excB, int nexcB,
                           const double *g, int M, const double2 *C, double2 *S, int64_t nsa,
                           int64_t nsb, hipStream_t st) {
    const int lds_max = g_lds_max > 0 ? g_lds_max : 65536;
    const int64_t per = nsb * (int64_t)sizeof(double2) + (int64_t)M * M * (int64_t)sizeof(double);
    int64_t ec = per > 0 ? lds_max / per : 0;
    if (ec > nexcA) ec = nexcA;
    if (ec > 16) ec = 16;
    if (ec >= 1) {
        const size_t shm = (size_t)(ec * per);
        hipLaunchKernelGGL(k_sigma_ab_lds, dim3((unsigned)nsa), dim3(512), shm, st, excA, nexcA, excB,
                           nexcB, g, M, C, S, nsb, (int)ec);
        return hipGetLastError();
    }
    if (nexcA > kMaxExc) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sigma_ab, dim3((unsigned)nsa), dim3(256), 0, st, excA, nexcA, excB, nexcB, g, M, C, S, nsb);
    return hipGetLastError();
}

hipError_t launch_transpose(const double2 *in, double2 *out, int64_t rows, int64_t cols,
                            hipStream_t st) {
    const dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
    hipLaunchKernelGGL(k_transpose, grid, dim3(32, 8), 0, st, in, out, rows, cols);
    return hipGetLastError();
}

unsigned combine_grid(int64_t dim) {
    const unsigned b = blocks_for(dim, 256);
    return b > 1024 ? 1024 : b;
}

hipError_t launch_combine(double2 *S, const double2 *ST, const double2 *C, double ecore,
                          int64_t nsa, int64_t nsb, double *partial, hipStream_t st) {
    const unsigned grid = combine_grid(nsa * nsb);
    hipLaunchKernelGGL(k_combine, dim3(grid), dim3(256), 0, st, S, ST, C, ecore, nsa, nsb, partial);
    return hipGetLastError();
}

hipError_t launch_rdm_overlap(const double2 *A, int64_t nrows, int64_t ncols,
                              const uint32_t *exc, int nexc, double2 *O, hipStream_t st) {
    hipLaunchKernelGGL(k_rdm_overlap, dim3((unsigned)nrows), dim3(256), 0, st, A, ncols, exc, nexc, O);
    return hipGetLastError();
}

int cadj_blocks(const PairOp &op, int64_t nsa, int64_t nsb) {
    const CGrid g = cgrid_of(op, nsa, nsb);
    return (int)(g.gx * g.gy);
}

hipError_t launch_crot(int precision, void *psi, const PairOp &op, const uint32_t *lists,
                       const double *cs, int k, int64_t nsa, int64_t nsb, hipStream_t st) {
    const CGrid g = cgrid_of(op, nsa, nsb);
    if (precision == 0)
        hipLaunchKernelGGL(k_crot<double>, dim3(g.gx, g.gy), dim3(g.block), 0, st, (double2 *)psi, op, lists, cs, k, nsa, nsb);
    else
        hipLaunchKernelGGL(k_crot<float>, dim3(g.gx, g.gy), dim3(g.block), 0, st, (float2 *)psi, op, lists, cs, k, nsa, nsb);
    return hipGetLastError();
}

hipError_t launch_cadj(int precision, void *psi, void *lam, const PairOp &op, const uint32_t *lists,
                       const double *cs, int k, int64_t nsa, int64_t nsb, double *partial,
                       hipStream_t st) {
    const CGrid g = cgrid_of(op, nsa, nsb);
    if (precision == 0)
        hipLaunchKernelGGL(k_cadj<double>, dim3(g.gx, g.gy), dim3(g.block), 0, st, (double2 *)psi,
                           (double2 *)lam, op, lists, cs, k, nsa, nsb, partial);
    else
        hipLaunchKernelGGL(k_cadj<float>, dim3(g.gx, g.gy), dim3(g.block), 0, st, (float2 *)psi,
                           (float2 *)lam, op, lists, cs, k, nsa, nsb, partial);
    return hipGetLastError();
}

hipError_t launch_cvt(bool to_double, const void *in, void *out, int64_t n, hipStream_t st) {
    const unsigned grid = blocks_for(n, 256);
    if (to_double)
        hipLaunchKernelGGL(k_cvt_f2d, dim3(grid), dim3(256), 0, st, (const float2 *)in, (double2 *)out, n);
    else
        hipLaunchKernelGGL(k_cvt_d2f, dim3(grid), dim3(256), 0, st, (const double2 *)in, (float2 *)out, n);
    return hipGetLastError();
}

hipError_t launch_rdm_bin(const double2 *O, const int32_t *off, const int32_t *idx, int nbins,
                          double2 *out, hipStream_t st) {
    hipLaunchKernelGGL(k_rdm_bin, dim3(nbins), dim3(256), 0, st, O, off, idx, out);
    return hipGetLastError();
}

}  // namespace fsv
