// Kernels of the sector-compressed state C[Ia][Ib] (alpha-string-first
// product basis): excitation rotations and the adjoint step over alpha x beta
// pair lists, the Hamiltonian product H C, and conversions.  Every kernel is
// templated on the stored amplitude: complex or real, FP64 or FP32.  A state
// built from the reference with real angles and real integrals is exactly
// real, which halves every byte and flop of the energy/gradient pass.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <rocblas/rocblas.h>

#include <cstdlib>
#include <vector>

#include "fsv_device.h"
#include "fsv_internal.h"

namespace fsv {

namespace {

// ---- amplitude arithmetic (accumulations in FP64) ----
template <typename V> struct Vt;
template <> struct Vt<double2> { using R = double; using A = double2; };
template <> struct Vt<float2> { using R = float; using A = double2; };
template <> struct Vt<double> { using R = double; using A = double; };
template <> struct Vt<float> { using R = float; using A = double; };

// (a, b) <- (c a - s b, c b + s a)
__device__ __forceinline__ void rot(double &a, double &b, double c, double s) {
    const double t = a;
    a = c * a - s * b;
    b = c * b + s * t;
}
__device__ __forceinline__ void rot(float &a, float &b, float c, float s) {
    const float t = a;
    a = c * a - s * b;
    b = c * b + s * t;
}
__device__ __forceinline__ void rot(double2 &a, double2 &b, double c, double s) {
    rot(a.x, b.x, c, s);
    rot(a.y, b.y, c, s);
}
__device__ __forceinline__ void rot(float2 &a, float2 &b, float c, float s) {
    rot(a.x, b.x, c, s);
    rot(a.y, b.y, c, s);
}
// Re(conj(l) p)
__device__ __forceinline__ double dotre(double l, double p) { return l * p; }
__device__ __forceinline__ double dotre(float l, float p) { return (double)l * p; }
__device__ __forceinline__ double dotre(double2 l, double2 p) { return l.x * p.x + l.y * p.y; }
__device__ __forceinline__ double dotre(float2 l, float2 p) { return (double)l.x * p.x + (double)l.y * p.y; }
// acc += w x
__device__ __forceinline__ void axpy(double &acc, double w, double x) { acc += w * x; }
__device__ __forceinline__ void axpy(double2 &acc, double w, double2 x) {
    acc.x += w * x.x;
    acc.y += w * x.y;
}
template <typename A> __device__ __forceinline__ A zero();
template <> __device__ __forceinline__ double zero<double>() { return 0.0; }
template <> __device__ __forceinline__ double2 zero<double2>() { return make_double2(0.0, 0.0); }
__device__ __forceinline__ double neg_if(bool n, double v) { return n ? -v : v; }
__device__ __forceinline__ double2 neg_if(bool n, double2 v) { return n ? make_double2(-v.x, -v.y) : v; }
__device__ __forceinline__ double add(double a, double b) { return a + b; }
__device__ __forceinline__ double2 add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }

// ---- conversions ----
__device__ __forceinline__ void cvt(double a, double &b) { b = a; }
__device__ __forceinline__ void cvt(double a, float &b) { b = (float)a; }
__device__ __forceinline__ void cvt(float a, double &b) { b = a; }
__device__ __forceinline__ void cvt(double a, double2 &b) { b = make_double2(a, 0.0); }
__device__ __forceinline__ void cvt(double2 a, double2 &b) { b = a; }
__device__ __forceinline__ void cvt(double2 a, float2 &b) { b = make_float2((float)a.x, (float)a.y); }
__device__ __forceinline__ void cvt(float2 a, double2 &b) { b = make_double2(a.x, a.y); }
__device__ __forceinline__ void cvt(double2 a, double &b) { b = a.x; }

template <typename I, typename O>
__global__ void k_convert(const I *__restrict__ in, O *__restrict__ out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        cvt(in[i], out[i]);
}

// ------------------------------------------------------------ rotations ----
struct CGrid {
    unsigned gx, gy, block;
};

inline CGrid cgrid_of(const PairOp &op, int64_t nsa, int64_t nsb) {
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

// Alpha pair u of the operator (row u when it has no alpha part).
__device__ __forceinline__ void pair_row(const PairOp &op, const uint32_t *__restrict__ lists,
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

// Beta pair v (column v when it has no beta part).
__device__ __forceinline__ void pair_col(const PairOp &op, const uint32_t *__restrict__ lists,
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

template <typename V>
__global__ __launch_bounds__(256) void k_crot(V *__restrict__ psi, PairOp op,
                                              const uint32_t *__restrict__ lists,
                                              const double *__restrict__ cs, int k, int64_t nsa,
                                              int64_t nsb) {
    using R = typename Vt<V>::R;
    const R c = (R)cs[2 * k], s = (R)cs[2 * k + 1];
    const int64_t na = op.nA >= 0 ? op.nA : nsa, nb = op.nB >= 0 ? op.nB : nsb;
    for (int64_t u = blockIdx.y; u < na; u += gridDim.y) {
        int64_t ia, ia2;
        bool nrow;
        pair_row(op, lists, u, ia, ia2, nrow);
        for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nb;
             v += (int64_t)gridDim.x * blockDim.x) {
            int64_t ib, ib2;
            bool neg = nrow;
            pair_col(op, lists, v, ib, ib2, neg);
            const int64_t xs = ia * nsb + ib, xd = ia2 * nsb + ib2;
            V a = psi[xs], b = psi[xd];
            rot(a, b, c, neg ? -s : s);
            psi[xs] = a;
            psi[xd] = b;
        }
    }
}

// Partial of Re<lam|T|psi> over the operator's pairs, then psi, lam <- U^+ psi, U^+ lam.
template <typename V>
__global__ __launch_bounds__(256) void k_cadj(V *__restrict__ psi, V *__restrict__ lam, PairOp op,
                                              const uint32_t *__restrict__ lists,
                                              const double *__restrict__ cs, int k, int64_t nsa,
                                              int64_t nsb, double *__restrict__ partial) {
    using R = typename Vt<V>::R;
    const R c = (R)cs[2 * k], s = (R)cs[2 * k + 1];
    const int64_t na = op.nA >= 0 ? op.nA : nsa, nb = op.nB >= 0 ? op.nB : nsb;
    double acc = 0.0;
    for (int64_t u = blockIdx.y; u < na; u += gridDim.y) {
        int64_t ia, ia2;
        bool nrow;
        pair_row(op, lists, u, ia, ia2, nrow);
        for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nb;
             v += (int64_t)gridDim.x * blockDim.x) {
            int64_t ib, ib2;
            bool neg = nrow;
            pair_col(op, lists, v, ib, ib2, neg);
            const int64_t xs = ia * nsb + ib, xd = ia2 * nsb + ib2;
            V a = psi[xs], b = psi[xd], la = lam[xs], lb = lam[xd];
            const double o = dotre(lb, a) - dotre(la, b);
            acc += neg ? -o : o;
            const R sg = neg ? s : -s;  // U^+ = U(-theta)
            rot(a, b, c, sg);
            rot(la, lb, c, sg);
            psi[xs] = a;
            psi[xd] = b;
            lam[xs] = la;
            lam[xd] = lb;
        }
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = acc;
}

// The adjoint sweep on real states keeps psi and lam of each sector amplitude
// side by side, z[i] = (psi[i], lam[i]), so that one access moves both.
template <typename R> struct Zip2;
template <> struct Zip2<double> { using P = double2; };
template <> struct Zip2<float> { using P = float2; };

template <typename R>
__global__ __launch_bounds__(256) void k_zip(const R *__restrict__ psi, const R *__restrict__ lam,
                                             typename Zip2<R>::P *__restrict__ z, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        z[i] = {psi[i], lam[i]};
}

// k_cadj on the interleaved pairs.
template <typename R>
__global__ __launch_bounds__(256) void k_cadj_zip(typename Zip2<R>::P *__restrict__ z, PairOp op,
                                                  const uint32_t *__restrict__ lists,
                                                  const double *__restrict__ cs, int k, int64_t nsa,
                                                  int64_t nsb, double *__restrict__ partial) {
    const R c = (R)cs[2 * k], s = (R)cs[2 * k + 1];
    const int64_t na = op.nA >= 0 ? op.nA : nsa, nb = op.nB >= 0 ? op.nB : nsb;
    double acc = 0.0;
    for (int64_t u = blockIdx.y; u < na; u += gridDim.y) {
        int64_t ia, ia2;
        bool nrow;
        pair_row(op, lists, u, ia, ia2, nrow);
        for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nb;
             v += (int64_t)gridDim.x * blockDim.x) {
            int64_t ib, ib2;
            bool neg = nrow;
            pair_col(op, lists, v, ib, ib2, neg);
            const int64_t xs = ia * nsb + ib, xd = ia2 * nsb + ib2;
            const auto A = z[xs], B = z[xd];
            R a = A.x, la = A.y, b = B.x, lb = B.y;
            const double o = (double)lb * (double)a - (double)la * (double)b;
            acc += neg ? -o : o;
            const R sg = neg ? s : -s;  // U^+ = U(-theta)
            rot(a, b, c, sg);
            rot(la, lb, c, sg);
            z[xs] = {a, la};
            z[xd] = {b, lb};
        }
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.y * gridDim.x + blockIdx.x] = acc;
}

// ---------------------------------------------------------------- sigma ----
// out[I][:] = sum_k val[k] in[col[k]][:].  Blocks are dispatched row-fastest
// over one column tile at a time (blockIdx.x = row, blockIdx.y = tile), so the
// workgroups in flight share the input rows of the same tile in L2.
template <typename A>
__global__ __launch_bounds__(256) void k_spmm(const int64_t *__restrict__ rowptr,
                                              const int32_t *__restrict__ col,
                                              const double *__restrict__ val, const A *__restrict__ in,
                                              A *__restrict__ out, int64_t ncols) {
    const int64_t I = blockIdx.x;
    const int64_t k0 = rowptr[I], k1 = rowptr[I + 1];
    const int64_t c = (int64_t)blockIdx.y * blockDim.x + threadIdx.x;
    if (c >= ncols) return;
    A acc = zero<A>();
    for (int64_t k = k0; k < k1; ++k) axpy(acc, val[k], in[(int64_t)col[k] * ncols + c]);
    out[I * ncols + c] = acc;
}

// Dense copy of a CSR matrix (one workgroup per row; columns within a row are
// distinct, so the scatter needs no ordering).
__global__ __launch_bounds__(256) void k_csr_dense(const int64_t *__restrict__ rowptr,
                                                   const int32_t *__restrict__ col,
                                                   const double *__restrict__ val, double *__restrict__ out,
                                                   int64_t n) {
    const int64_t I = blockIdx.x;
    double *row = out + I * n;
    for (int64_t c = threadIdx.x; c < n; c += blockDim.x) row[c] = 0.0;
    __syncthreads();
    for (int64_t k = rowptr[I] + threadIdx.x; k < rowptr[I + 1]; k += blockDim.x) row[col[k]] = val[k];
}

// Same-spin product on the matrix cores: out (rows x w*ncols, row-major) =
// H (rows x rows, row-major, symmetric) * in (rows x w*ncols), as the
// column-major product in' * H of rocBLAS (in' = in viewed column-major).
// Atomics stay disallowed on the handle, so the result is deterministic and no
// memset enters a captured graph.
hipError_t dense_same_spin(void *blas, const double *H, const double *in, double *out, int64_t rows,
                           int64_t wcols, hipStream_t st) {
    rocblas_handle h = (rocblas_handle)blas;
    const double one = 1.0, zero = 0.0;
    if (rocblas_set_stream(h, st) != rocblas_status_success) return hipErrorInvalidHandle;
    const rocblas_status rs = rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, (rocblas_int)wcols,
                                            (rocblas_int)rows, (rocblas_int)rows, &one, in, (rocblas_int)wcols, H,
                                            (rocblas_int)rows, &zero, out, (rocblas_int)wcols);
    return rs == rocblas_status_success ? hipSuccess : hipErrorLaunchFailure;
}

// Same-spin beta part of a real state accumulated in place, with no
// transposes of the state: S[Ia][Ib] += sum_Jb Hb[Ib][Jb] C[Ia][Jb].  Read
// column-major, the row-major S and C are nsb x nsa matrices and the
// row-major Hb^T (HbT) is Hb, so this is S += Hb x C, one untransposed GEMM.
hipError_t dense_beta_accumulate(void *blas, const double *HbT, const double *C, double *S, int64_t nsa,
                                 int64_t nsb, hipStream_t st) {
    rocblas_handle h = (rocblas_handle)blas;
    const double one = 1.0;
    if (rocblas_set_stream(h, st) != rocblas_status_success) return hipErrorInvalidHandle;
    const rocblas_status rs =
        rocblas_dgemm(h, rocblas_operation_none, rocblas_operation_none, (rocblas_int)nsb, (rocblas_int)nsa,
                      (rocblas_int)nsb, &one, HbT, (rocblas_int)nsb, C, (rocblas_int)nsb, &one, S, (rocblas_int)nsb);
    return rs == rocblas_status_success ? hipSuccess : hipErrorLaunchFailure;
}

// Alpha-beta two-body term, one workgroup per output row Ia:
//   S[Ia][Ib] += sum_{e in exc(Ia)} sum_{f in exc(Ib)} s_e s_f (pq_e|rs_f) C[J_e][J_f].
// The alpha excitations are taken ec at a time.  Their source rows are staged
// in LDS interleaved as Rt[Jb][e] and their weights as Wt[rs][e] = s_e (pq_e|rs),
// so each beta excitation of a thread's Ib costs one contiguous LDS read of
// the ec row values and one of the ec weights.
template <typename A>
__global__ __launch_bounds__(512) void k_sigma_ab(const uint32_t *__restrict__ excA, int nexcA,
                                                  const uint32_t *__restrict__ excB, int nexcB,
                                                  const double *__restrict__ g, int M,
                                                  const A *__restrict__ C, A *__restrict__ S,
                                                  int64_t nsb, int ec) {
    extern __shared__ double smem_d[];
    A *Rt = (A *)smem_d;                           // nsb * ec
    double *Wt = (double *)(Rt + (int64_t)nsb * ec);  // M2 * ec
    const int64_t Ia = blockIdx.x;
    const int M2 = M * M;
    for (int e0 = 0; e0 < nexcA; e0 += ec) {
        const int ne = min(ec, nexcA - e0);
        for (int e = 0; e < ne; ++e) {
            const uint32_t w = excA[Ia * nexcA + e0 + e];
            const int64_t Ja = w & 0xFFFFu;
            const int pq = (w >> 16) & 0x1FFu;
            const double sa = (w >> 31) ? -1.0 : 1.0;
            for (int64_t jb = threadIdx.x; jb < nsb; jb += blockDim.x) Rt[jb * ec + e] = C[Ja * nsb + jb];
            for (int rs = threadIdx.x; rs < M2; rs += blockDim.x) Wt[rs * ec + e] = sa * g[pq * M2 + rs];
        }
        __syncthreads();
        for (int64_t Ib = threadIdx.x; Ib < nsb; Ib += blockDim.x) {
            A acc = zero<A>();
            for (int f = 0; f < nexcB; ++f) {
                const uint32_t eb = excB[Ib * nexcB + f];
                const A *r = Rt + (int64_t)(eb & 0xFFFFu) * ec;
                const double *wr = Wt + (int)((eb >> 16) & 0x1FFu) * ec;
                A t = zero<A>();
                for (int e = 0; e < ne; ++e) axpy(t, wr[e], r[e]);
                acc = add(acc, neg_if((eb >> 31) != 0, t));
            }
            S[Ia * nsb + Ib] = add(S[Ia * nsb + Ib], acc);
        }
        __syncthreads();
    }
}

// Same term with each thread's beta-excitation list held in registers: a
// workgroup of 1024 threads takes the output columns Ib in groups of 1024;
// for each group it loads every thread's (J_f, rs_f, s_f) list once, then
// streams the alpha excitations through LDS ec at a time.  The list is read
// once per output element instead of once per LDS chunk.  MAXF bounds the
// number of beta excitations per string (N (M - N + 1)).
template <typename A, int MAXF, int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_sigma_ab_reg(const uint32_t *__restrict__ excA, int nexcA,
                                                       const uint32_t *__restrict__ excB, int nexcB,
                                                       const double *__restrict__ g, int M,
                                                       const A *__restrict__ C, A *__restrict__ S,
                                                       int64_t nsb, int ec) {
    extern __shared__ double smem_d[];
    A *Rt = (A *)smem_d;                              // nsb * ec
    double *Wt = (double *)(Rt + (int64_t)nsb * ec);  // M2 * ec
    const int64_t Ia = blockIdx.x;
    const int M2 = M * M;
    for (int64_t ib0 = 0; ib0 < nsb; ib0 += blockDim.x) {
        const int64_t Ib = ib0 + threadIdx.x;
        const bool active = Ib < nsb;
        uint32_t ex[MAXF];
#pragma unroll
        for (int f = 0; f < MAXF; ++f) ex[f] = (active && f < nexcB) ? excB[Ib * nexcB + f] : 0u;
        A acc = zero<A>();
        for (int e0 = 0; e0 < nexcA; e0 += ec) {
            const int ne = min(ec, nexcA - e0);
            __syncthreads();  // previous chunk fully consumed
            for (int e = 0; e < ne; ++e) {
                const uint32_t w = excA[Ia * nexcA + e0 + e];
                const int64_t Ja = w & 0xFFFFu;
                const int pq = (w >> 16) & 0x1FFu;
                const double sa = (w >> 31) ? -1.0 : 1.0;
                for (int64_t jb = threadIdx.x; jb < nsb; jb += blockDim.x) Rt[jb * ec + e] = C[Ja * nsb + jb];
                for (int rs = threadIdx.x; rs < M2; rs += blockDim.x) Wt[rs * ec + e] = sa * g[pq * M2 + rs];
            }
            __syncthreads();
            if (active) {
#pragma unroll
                for (int f = 0; f < MAXF; ++f) {
                    if (f < nexcB) {
                        const uint32_t eb = ex[f];
                        const A *r = Rt + (int64_t)(eb & 0xFFFFu) * ec;
                        const double *wr = Wt + (int)((eb >> 16) & 0x1FFu) * ec;
                        A t = zero<A>();
                        for (int e = 0; e < ne; ++e) axpy(t, wr[e], r[e]);
                        acc = add(acc, neg_if((eb >> 31) != 0, t));
                    }
                }
            }
        }
        if (active) S[Ia * nsb + Ib] = add(S[Ia * nsb + Ib], acc);
    }
}

// Factorised alpha-beta term, (pq|rs) = sum_l L_l[pq] L_l[rs] (l < R, padded
// to RP = 8 with zero columns of Lt, which is M^2 x RP; wider ranks take the
// direct product):
//   S[Ia][Ib] += sum_l (A_l C B_l^T)[Ia][Ib],  A_l = sum_pq L_l[pq] E^alpha_pq,
//   B_l = sum_rs L_l[rs] E^beta_rs,
// in two steps through Y[Ia][Jb][l] = (A_l C)[Ia][Jb] (l fastest).
//
// Step 1 gathers whole rows of C: a workgroup is one alpha string Ia and 256
// beta strings Jb, so Ia's excitation list and the factor row of each
// excitation are workgroup-uniform and every coalesced load of C feeds RP
// multiply-adds.
template <typename A, int RP>
__global__ __launch_bounds__(256) void k_lr_a(const A *__restrict__ C, A *__restrict__ Y,
                                              const uint32_t *__restrict__ excA, int nexcA,
                                              const double *__restrict__ Lt, int64_t nsb) {
    const int64_t Ia = blockIdx.x;
    const int64_t Jb = (int64_t)blockIdx.y * blockDim.x + threadIdx.x;
    const bool active = Jb < nsb;
    const int64_t jb = active ? Jb : nsb - 1;
    const uint32_t *ex = excA + Ia * nexcA;
    A acc[RP];
#pragma unroll
    for (int l = 0; l < RP; ++l) acc[l] = zero<A>();
    int e = 0;
    for (; e + 4 <= nexcA; e += 4) {
        A x[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) x[u] = C[(int64_t)(ex[e + u] & 0xFFFFu) * nsb + jb];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const uint32_t ea = ex[e + u];
            const double *lr = Lt + ((ea >> 16) & 0x1FFu) * RP;
            const A xv = neg_if((ea >> 31) != 0, x[u]);
#pragma unroll
            for (int l = 0; l < RP; ++l) axpy(acc[l], lr[l], xv);
        }
    }
    for (; e < nexcA; ++e) {
        const uint32_t ea = ex[e];
        const double *lr = Lt + ((ea >> 16) & 0x1FFu) * RP;
        const A xv = neg_if((ea >> 31) != 0, C[(int64_t)(ea & 0xFFFFu) * nsb + jb]);
#pragma unroll
        for (int l = 0; l < RP; ++l) axpy(acc[l], lr[l], xv);
    }
    if (active) {
        A *y = Y + (Ia * nsb + Jb) * RP;
#pragma unroll
        for (int l = 0; l < RP; ++l) y[l] = acc[l];
    }
}

// Doubles of k_lr_b's staged factor rows (M2 rows of ws), rounded up to an
// even count so that the intermediate rows after them start 16-byte aligned
// (complex rows are read as 16-byte values).
__host__ __device__ inline size_t lr_lt_words(int M2, int ws) { return ((size_t)M2 * ws + 1) & ~(size_t)1; }

constexpr int kExcBatch = 8;    // beta-list words loaded together in the step-2 loop of k_lr_b
constexpr int kExcBatchAB = 4;  // and of k_lr_ab (which must stay within 64 VGPRs: two workgroups per CU)

// Step 2, row-local: S[Ia][Ib] += sum_{f in exc(Ib)} s_f sum_l L_l[rs_f]
// Y[Ia][Jb_f][l].  One workgroup per Ia stages its Y row (nsb x lc values)
// and the matching lc columns of Lt in LDS, lc of the RP values at a time;
// the beta lists are read transposed (excBT[f][Ib]) so the lanes' loads
// coalesce.  The staged rows are ys (Y) and ws (Lt) elements apart: with
// lc = 8 a 64-byte stride would start every lane's 16-byte LDS read in one
// of only 4 bank groups, so the host pads the strides by 16 bytes.
template <typename A>
__global__ __launch_bounds__(1024) void k_lr_b(const A *__restrict__ Y, A *__restrict__ S,
                                               const uint32_t *__restrict__ excBT, int nexcB,
                                               const double *__restrict__ Lt, int M2, int RP, int64_t nsb,
                                               int lc, int ys, int ws) {
    extern __shared__ double smem_d[];
    double *lt = smem_d;               // M2 x ws
    A *yr = (A *)(lt + lr_lt_words(M2, ws));  // nsb x ys, 16-byte aligned
    const int64_t Ia = blockIdx.x;
    const A *yrow = Y + Ia * nsb * RP;
    A *srow = S + Ia * nsb;
    for (int l0 = 0; l0 < RP; l0 += lc) {
        __syncthreads();  // readers of the previous chunk are done
        for (int i = threadIdx.x; i < M2 * lc; i += blockDim.x)
            lt[(i / lc) * ws + i % lc] = Lt[(i / lc) * RP + l0 + i % lc];
        for (int64_t i = threadIdx.x; i < nsb * lc; i += blockDim.x)
            yr[(i / lc) * ys + i % lc] = yrow[(i / lc) * RP + l0 + i % lc];
        __syncthreads();
        for (int64_t Ib = threadIdx.x; Ib < nsb; Ib += blockDim.x) {
            A acc = zero<A>();
            auto step = [&](uint32_t eb) {
                const double *w = lt + ((eb >> 16) & 0x1FFu) * ws;
                const A *y = yr + (int64_t)(eb & 0xFFFFu) * ys;
                A t = zero<A>();
                for (int l = 0; l < lc; ++l) axpy(t, w[l], y[l]);
                acc = add(acc, neg_if((eb >> 31) != 0, t));
            };
            int f = 0;
            for (; f + kExcBatch <= nexcB; f += kExcBatch) {  // the list words in flight together
                uint32_t eb[kExcBatch];
#pragma unroll
                for (int u = 0; u < kExcBatch; ++u) eb[u] = excBT[(int64_t)(f + u) * nsb + Ib];
#pragma unroll
                for (int u = 0; u < kExcBatch; ++u) step(eb[u]);
            }
            for (; f < nexcB; ++f) step(excBT[(int64_t)f * nsb + Ib]);
            srow[Ib] = add(srow[Ib], acc);
        }
    }
}

// Both steps in one workgroup per alpha string Ia (real states, RP = 8, the
// Y row in LDS): the row Y[Ia][:][:] is built from Ia's alpha excitations
// (each thread one Jb; the excitation words and factor rows are
// workgroup-uniform, so they come through scalar loads) straight into LDS,
// then step 2 runs on it as in k_lr_b.  Y never goes to memory.  Rows are
// kLrStride = 9 doubles apart (72 bytes: lanes' 8-byte reads start in 32
// different bank pairs), which keeps two workgroups per CU at 24 qubits.
// A string's diagonal excitations (the last ndA / ndB entries of its list)
// all map it to itself, so each step takes them as one term with the
// string's summed factor row (da / db).
constexpr int kLrStride = 9;

__global__ __launch_bounds__(1024) void k_lr_ab(const double *__restrict__ C, double *__restrict__ S,
                                                const uint32_t *__restrict__ excA, int nexcA,
                                                const uint32_t *__restrict__ excBT, int nexcB,
                                                const double *__restrict__ Lt, int M2, int64_t nsb,
                                                const double *__restrict__ da, const double *__restrict__ db,
                                                int ndA, int ndB) {
    constexpr int RP = 8;
    extern __shared__ double smem_d[];
    double *lt = smem_d;                // M2 x kLrStride
    double *yr = lt + M2 * kLrStride;   // nsb x kLrStride
    const int64_t Ia = blockIdx.x;
    for (int i = threadIdx.x; i < M2 * RP; i += blockDim.x) lt[(i / RP) * kLrStride + i % RP] = Lt[i];
    const uint32_t *ex = excA + Ia * nexcA;
    const int noffA = nexcA - ndA, noffB = nexcB - ndB;
    const double *dar = da + Ia * RP;
    for (int64_t Jb = threadIdx.x; Jb < nsb; Jb += blockDim.x) {
        double acc[RP];
        {
            const double xv = C[Ia * nsb + Jb];
#pragma unroll
            for (int l = 0; l < RP; ++l) acc[l] = dar[l] * xv;
        }
        int e = 0;
        for (; e + 4 <= noffA; e += 4) {
            double x[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) x[u] = C[(int64_t)(ex[e + u] & 0xFFFFu) * nsb + Jb];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint32_t ea = ex[e + u];
                const double *lr = Lt + ((ea >> 16) & 0x1FFu) * RP;
                const double xv = neg_if((ea >> 31) != 0, x[u]);
#pragma unroll
                for (int l = 0; l < RP; ++l) axpy(acc[l], lr[l], xv);
            }
        }
        for (; e < noffA; ++e) {
            const uint32_t ea = ex[e];
            const double *lr = Lt + ((ea >> 16) & 0x1FFu) * RP;
            const double xv = neg_if((ea >> 31) != 0, C[(int64_t)(ea & 0xFFFFu) * nsb + Jb]);
#pragma unroll
            for (int l = 0; l < RP; ++l) axpy(acc[l], lr[l], xv);
        }
#pragma unroll
        for (int l = 0; l < RP; ++l) yr[Jb * kLrStride + l] = acc[l];
    }
    __syncthreads();
    double *srow = S + Ia * nsb;
    for (int64_t Ib = threadIdx.x; Ib < nsb; Ib += blockDim.x) {
        double acc = 0.0;
        {
            const double *dbr = db + Ib * RP;
            const double *y = yr + Ib * kLrStride;
#pragma unroll
            for (int l = 0; l < RP; ++l) axpy(acc, dbr[l], y[l]);
        }
        auto step = [&](uint32_t eb) {
            const double *w = lt + ((eb >> 16) & 0x1FFu) * kLrStride;
            const double *y = yr + (int64_t)(eb & 0xFFFFu) * kLrStride;
            double t = 0.0;
#pragma unroll
            for (int l = 0; l < RP; ++l) axpy(t, w[l], y[l]);
            acc += neg_if((eb >> 31) != 0, t);
        };
        int f = 0;
        for (; f + kExcBatchAB <= noffB; f += kExcBatchAB) {
            uint32_t eb[kExcBatchAB];
#pragma unroll
            for (int u = 0; u < kExcBatchAB; ++u) eb[u] = excBT[(int64_t)(f + u) * nsb + Ib];
#pragma unroll
            for (int u = 0; u < kExcBatchAB; ++u) step(eb[u]);
        }
        for (; f < noffB; ++f) step(excBT[(int64_t)f * nsb + Ib]);
        srow[Ib] += acc;
    }
}

// ------------------------------------------------------------ screening ----
// ADAPT pool screening, one launch for the whole pool: workgroup (x, t)
// accumulates, over its share of pool operator t's pairs, the real part of
// <lam| T_t |psi> = sum s (lam[x'] psi[x] - lam[x] psi[x']); psi and lam are
// only read.  partial[t * gridDim.x + x].
template <typename V>
__global__ __launch_bounds__(256) void k_pool(const V *__restrict__ psi, const V *__restrict__ lam,
                                              const PairOp *__restrict__ ops,
                                              const uint32_t *__restrict__ lists, int64_t nsa, int64_t nsb,
                                              double *__restrict__ partial) {
    const PairOp op = ops[blockIdx.y];
    const uint32_t na = (uint32_t)(op.nA >= 0 ? op.nA : nsa), nb = (uint32_t)(op.nB >= 0 ? op.nB : nsb);
    const uint32_t np = na * nb;
    double acc = 0.0;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < np; t += gridDim.x * blockDim.x) {
        const uint32_t u = t / nb, v = t - u * nb;
        int64_t ia, ia2, ib, ib2;
        bool neg;
        pair_row(op, lists, u, ia, ia2, neg);
        pair_col(op, lists, v, ib, ib2, neg);
        const int64_t xs = ia * nsb + ib, xd = ia2 * nsb + ib2;
        const double o = dotre(lam[xd], psi[xs]) - dotre(lam[xs], psi[xd]);
        acc += neg ? -o : o;
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = acc;
}

// Same term without LDS staging (rows too long for LDS): gathers from global.
template <typename A>
__global__ __launch_bounds__(256) void k_sigma_ab_global(const uint32_t *__restrict__ excA, int nexcA,
                                                         const uint32_t *__restrict__ excB, int nexcB,
                                                         const double *__restrict__ g, int M,
                                                         const A *__restrict__ C, A *__restrict__ S,
                                                         int64_t nsb) {
    const int64_t Ia = blockIdx.x;
    const int M2 = M * M;
    for (int64_t Ib = threadIdx.x; Ib < nsb; Ib += blockDim.x) {
        A acc = zero<A>();
        for (int e = 0; e < nexcA; ++e) {
            const uint32_t w = excA[Ia * nexcA + e];
            const int64_t Ja = w & 0xFFFFu;
            const double *gp = g + ((w >> 16) & 0x1FFu) * M2;
            A t = zero<A>();
            for (int f = 0; f < nexcB; ++f) {
                const uint32_t eb = excB[Ib * nexcB + f];
                const double gv = gp[(eb >> 16) & 0x1FFu];
                axpy(t, (eb >> 31) ? -gv : gv, C[Ja * nsb + (eb & 0xFFFFu)]);
            }
            acc = add(acc, neg_if((w >> 31) != 0, t));
        }
        S[Ia * nsb + Ib] = add(S[Ia * nsb + Ib], acc);
    }
}

template <typename A>
__global__ void k_transpose(const A *__restrict__ in, A *__restrict__ out, int64_t rows, int64_t cols) {
    __shared__ A t[32][33];
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

// S[Ia][Ib] += ST[Ib][Ia] + ecore C[Ia][Ib]; per-block partials of Re<C|S>.
// The transposed operand is read through an LDS tile.
template <typename A>
__global__ void k_combine(A *__restrict__ S, const A *__restrict__ ST, const A *__restrict__ C,
                          double ecore, int64_t nsa, int64_t nsb, double *__restrict__ partial) {
    __shared__ A t[32][33];
    double acc = 0.0;
    const int64_t tiles_b = (nsb + 31) / 32, tiles = ((nsa + 31) / 32) * tiles_b;
    for (int64_t tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
        const int64_t a0 = (tile / tiles_b) * 32, b0 = (tile % tiles_b) * 32;
        for (int j = threadIdx.y; j < 32; j += blockDim.y) {  // ST rows b0+j, columns a0+x
            const int64_t ib = b0 + j, ia = a0 + threadIdx.x;
            if (ib < nsb && ia < nsa) t[j][threadIdx.x] = ST[ib * nsa + ia];
        }
        __syncthreads();
        for (int j = threadIdx.y; j < 32; j += blockDim.y) {
            const int64_t ia = a0 + j, ib = b0 + threadIdx.x;
            if (ia < nsa && ib < nsb) {
                const A c = C[ia * nsb + ib];
                A s = S[ia * nsb + ib];
                s = add(s, t[threadIdx.x][j]);
                axpy(s, ecore, c);
                S[ia * nsb + ib] = s;
                acc += dotre(c, s);
            }
        }
        __syncthreads();
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0 && threadIdx.y == 0) partial[blockIdx.x] = acc;
}

// String Hamiltonian values from their two-body parts and the one-body
// descriptors (see launch_string_h_values).
__global__ __launch_bounds__(256) void k_string_h_values(double *__restrict__ val, const double *__restrict__ v2,
                                                         const int32_t *__restrict__ desc,
                                                         const uint32_t *__restrict__ str,
                                                         const double *__restrict__ ht, int M, int64_t n) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t d = desc[e];
        double o = 0.0;
        if (d <= -2) {
            const uint32_t s = str[-2 - d];
            for (int i = 0; i < M; ++i)
                if (s >> i & 1u) o += ht[i * M + i];
        } else if (d >= 0) {
            o = ht[d & 0x3FFFFFFF];
            if (d & (1 << 30)) o = -o;
        }
        val[e] = o + v2[e];
    }
}

// S += ecore C and this workgroup's share of <C|S> (real states whose beta
// part went straight into S).
__global__ __launch_bounds__(256) void k_ecore_dot(double *__restrict__ S, const double *__restrict__ C, double ecore,
                                                   int64_t dim, double *__restrict__ partial) {
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim; i += (int64_t)gridDim.x * blockDim.x) {
        const double c = C[i];
        double s = S[i];
        axpy(s, ecore, c);
        S[i] = s;
        acc += c * s;
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

// k_ecore_dot for a real state whose adjoint sweep follows on (psi, lam)
// pairs: the pairs z[i] = (C[i], S[i] + ecore C[i]) are written instead of
// S, so that the sweep needs no separate interleaving pass.
__global__ __launch_bounds__(256) void k_ecore_zip(const double *__restrict__ S, const double *__restrict__ C,
                                                   double ecore, int64_t dim, double2 *__restrict__ z,
                                                   double *__restrict__ partial) {
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < dim; i += (int64_t)gridDim.x * blockDim.x) {
        const double c = C[i];
        double s = S[i];
        axpy(s, ecore, c);
        z[i] = make_double2(c, s);
        acc += c * s;
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) partial[blockIdx.x] = acc;
}

template <typename O>  // O = double2 or float2 (dense complex amplitude)
__global__ void k_scatter_real(O *__restrict__ lam,
                               const double *__restrict__ S, const uint64_t *__restrict__ Xa,
                               const uint64_t *__restrict__ Xb, const uint32_t *__restrict__ sa,
                               const uint32_t *__restrict__ PPb, int64_t nsb) {
    const int64_t Ia = blockIdx.y;
    for (int64_t Ib = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; Ib < nsb;
         Ib += (int64_t)gridDim.x * blockDim.x) {
        const uint64_t x = Xa[Ia] | Xb[Ib];
        const bool neg = popc(sa[Ia] & PPb[Ib]) & 1;
        const double v = S[Ia * nsb + Ib];
        lam[x].x = (decltype(lam->x))(neg ? -v : v);
        lam[x].y = (decltype(lam->x))0;
    }
}

int g_lds_max = -1;

// LDS chunk of the factor columns for step 2 (0: a row does not fit).
template <typename A>
int lr_chunk(const SectorTabs &T, int rp) {
    const size_t lim = g_lds_max > 0 ? (size_t)g_lds_max : 65536;
    const size_t per = (size_t)T.M * T.M * sizeof(double) + (size_t)T.nsb * sizeof(A);
    int lc = rp;
    while (lc > 0 && (size_t)lc * per + sizeof(double) > lim) lc >>= 1;  // + the alignment pad
    return lc;
}

// The one-kernel form applies to real states with RP = 8 whose LDS rows fit
// two workgroups per CU.
template <typename A, int RP>
bool lr_fused_ok(const SectorTabs &T) {
    if (sizeof(A) != sizeof(double) || RP != 8 || std::getenv("FSV_LR_SPLIT")) return false;
    return (size_t)(T.M * T.M + T.nsb) * kLrStride * sizeof(double) * 2 <= 163840 && g_lds_max >= 81920;
}

// Padded LDS strides (in elements) of k_lr_b's staged rows for lc values per
// row, when the padded rows still fit: 16 bytes more than the row for lc >= 4
// (16-byte reads); an odd number of doubles for real rows of lc < 4 (8-byte
// reads, 32 distinct bank pairs instead of 16).
template <typename A>
void lr_strides(const SectorTabs &T, int lc, int &ys, int &ws) {
    const size_t lim = g_lds_max > 0 ? (size_t)g_lds_max : 65536;
    ys = lc;
    ws = lc;
    if (lc < 4 && sizeof(A) != sizeof(double)) return;
    const int py = lc < 4 ? lc + 1 : lc + (int)(16 / sizeof(A)), pw = lc < 4 ? lc + 1 : lc + 2;
    if (lr_lt_words(T.M * T.M, pw) * sizeof(double) + (size_t)T.nsb * py * sizeof(A) <= lim) {
        ys = py;
        ws = pw;
    }
}

template <typename A, int RP>
hipError_t lr_launch(const SectorTabs &T, const A *C, A *S, hipStream_t st) {
    if (lr_fused_ok<A, RP>(T)) {
        const size_t shm = (size_t)(T.M * T.M + T.nsb) * kLrStride * sizeof(double);
        hipLaunchKernelGGL(k_lr_ab, dim3((unsigned)T.nsa), dim3(1024), shm, st, (const double *)C, (double *)S,
                           T.excA, T.nexcA, T.excBT, T.nexcB, T.Lt, T.M * T.M, T.nsb, T.lr_da, T.lr_db, T.ndA,
                           T.ndB);
        return hipGetLastError();
    }
    A *Y = (A *)T.YT;
    const int lc = lr_chunk<A>(T, RP);
    if (lc < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL((k_lr_a<A, RP>), dim3((unsigned)T.nsa, (unsigned)((T.nsb + 255) / 256)), dim3(256), 0, st,
                       C, Y, T.excA, T.nexcA, T.Lt, T.nsb);
    const int M2 = T.M * T.M;
    int ys, ws;
    lr_strides<A>(T, lc, ys, ws);
    const size_t shm = lr_lt_words(M2, ws) * sizeof(double) + (size_t)T.nsb * ys * sizeof(A);
    hipLaunchKernelGGL((k_lr_b<A>), dim3((unsigned)T.nsa), dim3(1024), shm, st, Y, S, T.excBT, T.nexcB, T.Lt, M2,
                       RP, T.nsb, lc, ys, ws);
    return hipGetLastError();
}

}  // namespace

bool lr_uses_intermediate(const SectorTabs &T, bool cplex) {
    if (T.R <= 0 || T.nexcA <= 0 || T.nexcB <= 0) return false;
    return cplex ? true : !lr_fused_ok<double, 8>(T);
}

namespace {

template <typename A>
hipError_t sigma_impl(const SectorTabs &T, const A *C, A *S, A *CT, A *ST, double *epart, hipStream_t st,
                      double2 *zout, bool *zipped) {
    const int64_t nsa = T.nsa, nsb = T.nsb;
    constexpr int64_t w = sizeof(A) / sizeof(double);  // doubles per amplitude
    // same-spin alpha part (with the alpha one-body terms): dense on the
    // matrix cores, or sparse rows
    if (T.ha_dense) {
        const hipError_t e = dense_same_spin(T.blas, T.ha_dense, (const double *)C, (double *)S, nsa, w * nsb, st);
        if (e != hipSuccess) return e;
    } else {
        hipLaunchKernelGGL(k_spmm<A>, dim3((unsigned)nsa, (unsigned)((nsb + 255) / 256)), dim3(256), 0, st,
                           T.ha_ptr, T.ha_col, T.ha_val, C, S, nsb);
    }
    // alpha-beta part, directly or through the factors of (pq|rs)
    if (T.nexcA > 0 && T.nexcB > 0 && T.R == 0) {
        const int lds = g_lds_max > 0 ? g_lds_max : 65536;
        const int64_t per = nsb * (int64_t)sizeof(A) + (int64_t)T.M * T.M * (int64_t)sizeof(double);
        int64_t ec = lds / per;
        if (ec > T.nexcA) ec = T.nexcA;
        const size_t shm = (size_t)(ec * per);
        // Register-resident lists pay off while each workgroup covers the row
        // in at most two column groups (the staged rows are reloaded per group).
        if (ec >= 1 && T.nexcB <= 48 && nsb <= 2048)
            hipLaunchKernelGGL((k_sigma_ab_reg<A, 48, 1024>), dim3((unsigned)nsa), dim3(1024), shm, st, T.excA,
                               T.nexcA, T.excB, T.nexcB, T.g, T.M, C, S, nsb, (int)ec);
        else if (ec >= 1 && T.nexcB <= 64 && nsb <= 1024)
            hipLaunchKernelGGL((k_sigma_ab_reg<A, 64, 512>), dim3((unsigned)nsa), dim3(512), shm, st, T.excA,
                               T.nexcA, T.excB, T.nexcB, T.g, T.M, C, S, nsb, (int)ec);
        else if (ec >= 1)
            hipLaunchKernelGGL(k_sigma_ab<A>, dim3((unsigned)nsa), dim3(512), shm, st, T.excA,
                               T.nexcA, T.excB, T.nexcB, T.g, T.M, C, S, nsb, (int)ec);
        else  // a source row does not fit in LDS
            hipLaunchKernelGGL(k_sigma_ab_global<A>, dim3((unsigned)nsa), dim3(256), 0, st, T.excA, T.nexcA,
                               T.excB, T.nexcB, T.g, T.M, C, S, nsb);
    }
    if (T.nexcA > 0 && T.nexcB > 0 && T.R > 0) {
        if (T.R > 8) return hipErrorInvalidValue;  // wider factorisations take the direct product
        const hipError_t e = lr_launch<A, 8>(T, C, S, st);
        if (e != hipSuccess) return e;
    }
    if (T.hb_dense_t && sizeof(A) == sizeof(double)) {
        // real state: the beta GEMM accumulates into S directly
        const hipError_t e = dense_beta_accumulate(T.blas, T.hb_dense_t, (const double *)C, (double *)S, nsa, nsb, st);
        if (e != hipSuccess) return e;
        if (zout) {
            hipLaunchKernelGGL(k_ecore_zip, dim3(combine_grid(nsa * nsb)), dim3(256), 0, st, (const double *)S,
                               (const double *)C, T.ecore, nsa * nsb, zout, epart);
            if (zipped) *zipped = true;
        } else {
            hipLaunchKernelGGL(k_ecore_dot, dim3(combine_grid(nsa * nsb)), dim3(256), 0, st, (double *)S,
                               (const double *)C, T.ecore, nsa * nsb, epart);
        }
        return hipGetLastError();
    }
    // same-spin beta part on the transpose, then combine
    {
        const dim3 grid((unsigned)((nsb + 31) / 32), (unsigned)((nsa + 31) / 32));
        hipLaunchKernelGGL(k_transpose<A>, grid, dim3(32, 8), 0, st, C, CT, nsa, nsb);
    }
    if (T.hb_dense) {
        const hipError_t e = dense_same_spin(T.blas, T.hb_dense, (const double *)CT, (double *)ST, nsb, w * nsa, st);
        if (e != hipSuccess) return e;
    } else {
        hipLaunchKernelGGL(k_spmm<A>, dim3((unsigned)nsb, (unsigned)((nsa + 255) / 256)), dim3(256), 0, st,
                           T.hb_ptr, T.hb_col, T.hb_val, CT, ST, nsa);
    }
    hipLaunchKernelGGL(k_combine<A>, dim3(combine_grid(nsa * nsb)), dim3(32, 8), 0, st, S, ST, C, T.ecore,
                       nsa, nsb, epart);
    return hipGetLastError();
}

template <typename V>
hipError_t crot_impl(void *psi, const PairOp &op, const uint32_t *lists, const double *cs, int k,
                     int64_t nsa, int64_t nsb, hipStream_t st) {
    const CGrid g = cgrid_of(op, nsa, nsb);
    hipLaunchKernelGGL(k_crot<V>, dim3(g.gx, g.gy), dim3(g.block), 0, st, (V *)psi, op, lists, cs, k, nsa, nsb);
    return hipGetLastError();
}

template <typename V>
hipError_t cadj_impl(void *psi, void *lam, const PairOp &op, const uint32_t *lists, const double *cs,
                     int k, int64_t nsa, int64_t nsb, double *partial, hipStream_t st) {
    const CGrid g = cgrid_of(op, nsa, nsb);
    hipLaunchKernelGGL(k_cadj<V>, dim3(g.gx, g.gy), dim3(g.block), 0, st, (V *)psi, (V *)lam, op, lists, cs,
                       k, nsa, nsb, partial);
    return hipGetLastError();
}

template <typename R>
hipError_t cadj_zip_impl(void *z, const PairOp &op, const uint32_t *lists, const double *cs, int k,
                         int64_t nsa, int64_t nsb, double *partial, hipStream_t st) {
    const CGrid g = cgrid_of(op, nsa, nsb);
    hipLaunchKernelGGL(k_cadj_zip<R>, dim3(g.gx, g.gy), dim3(g.block), 0, st, (typename Zip2<R>::P *)z, op,
                       lists, cs, k, nsa, nsb, partial);
    return hipGetLastError();
}

template <typename R>
hipError_t zip_impl(const void *psi, const void *lam, void *z, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL(k_zip<R>, dim3(blocks_for(n, 256)), dim3(256), 0, st, (const R *)psi, (const R *)lam,
                       (typename Zip2<R>::P *)z, n);
    return hipGetLastError();
}

template <typename I, typename O>
hipError_t convert_impl(const void *in, void *out, int64_t n, hipStream_t st) {
    hipLaunchKernelGGL((k_convert<I, O>), dim3(blocks_for(n, 256)), dim3(256), 0, st, (const I *)in, (O *)out, n);
    return hipGetLastError();
}

}  // namespace

void init_sigma_kernels() {
    if (g_lds_max > 0) return;
    g_lds_max = 65536;
    std::vector<const void *> fns = {(const void *)k_sigma_ab<double>, (const void *)k_sigma_ab<double2>,
                                     (const void *)k_sigma_ab_reg<double, 48, 1024>,
                                     (const void *)k_sigma_ab_reg<double2, 48, 1024>,
                                     (const void *)k_sigma_ab_reg<double, 64, 512>,
                                     (const void *)k_sigma_ab_reg<double2, 64, 512>,
                                     (const void *)k_lr_b<double>, (const void *)k_lr_b<double2>,
                                     (const void *)k_lr_ab};
    bool ok = true;
    for (const void *f : fns)
        ok = ok && hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 163840) == hipSuccess;
    if (ok) g_lds_max = 163840;  // a gfx950 CU's LDS
    (void)hipGetLastError();
}

unsigned combine_grid(int64_t dim) {
    const int64_t tiles = (dim + 1023) / 1024;  // upper bound on 32x32 tiles in use
    return (unsigned)(tiles < 1 ? 1 : (tiles > 1024 ? 1024 : tiles));
}

int cadj_blocks(const PairOp &op, int64_t nsa, int64_t nsb) {
    const CGrid g = cgrid_of(op, nsa, nsb);
    return (int)(g.gx * g.gy);
}

hipError_t launch_crot(int vt, void *psi, const PairOp &op, const uint32_t *lists, const double *cs,
                       int k, int64_t nsa, int64_t nsb, hipStream_t st) {
    switch (vt) {
    case V_C128: return crot_impl<double2>(psi, op, lists, cs, k, nsa, nsb, st);
    case V_C64: return crot_impl<float2>(psi, op, lists, cs, k, nsa, nsb, st);
    case V_F64: return crot_impl<double>(psi, op, lists, cs, k, nsa, nsb, st);
    default: return crot_impl<float>(psi, op, lists, cs, k, nsa, nsb, st);
    }
}

hipError_t launch_cadj(int vt, void *psi, void *lam, const PairOp &op, const uint32_t *lists,
                       const double *cs, int k, int64_t nsa, int64_t nsb, double *partial,
                       hipStream_t st) {
    switch (vt) {
    case V_C128: return cadj_impl<double2>(psi, lam, op, lists, cs, k, nsa, nsb, partial, st);
    case V_C64: return cadj_impl<float2>(psi, lam, op, lists, cs, k, nsa, nsb, partial, st);
    case V_F64: return cadj_impl<double>(psi, lam, op, lists, cs, k, nsa, nsb, partial, st);
    default: return cadj_impl<float>(psi, lam, op, lists, cs, k, nsa, nsb, partial, st);
    }
}

hipError_t launch_cadj_zip(int vt, void *z, const PairOp &op, const uint32_t *lists, const double *cs, int k,
                           int64_t nsa, int64_t nsb, double *partial, hipStream_t st) {
    if (vt == V_F64) return cadj_zip_impl<double>(z, op, lists, cs, k, nsa, nsb, partial, st);
    if (vt == V_F32) return cadj_zip_impl<float>(z, op, lists, cs, k, nsa, nsb, partial, st);
    return hipErrorInvalidValue;
}

hipError_t launch_zip(int vt, const void *psi, const void *lam, void *z, int64_t n, hipStream_t st) {
    if (vt == V_F64) return zip_impl<double>(psi, lam, z, n, st);
    if (vt == V_F32) return zip_impl<float>(psi, lam, z, n, st);
    return hipErrorInvalidValue;
}

hipError_t launch_convert(int vi, const void *in, int vo, void *out, int64_t n, hipStream_t st) {
    if (vi == V_F32 && vo == V_F64) return convert_impl<float, double>(in, out, n, st);
    if (vi == V_F64 && vo == V_F32) return convert_impl<double, float>(in, out, n, st);
    if (vi == V_C64 && vo == V_C128) return convert_impl<float2, double2>(in, out, n, st);
    if (vi == V_C128 && vo == V_C64) return convert_impl<double2, float2>(in, out, n, st);
    if (vi == V_F64 && vo == V_C128) return convert_impl<double, double2>(in, out, n, st);
    if (vi == V_C128 && vo == V_F64) return convert_impl<double2, double>(in, out, n, st);
    return hipErrorInvalidValue;
}

hipError_t launch_sector_sigma(bool cplex, const SectorTabs &T, const void *C, void *S, void *CT, void *ST,
                               double *epart, hipStream_t st, void *zout, bool *zipped) {
    if (zipped) *zipped = false;
    if (cplex)
        return sigma_impl<double2>(T, (const double2 *)C, (double2 *)S, (double2 *)CT, (double2 *)ST, epart, st,
                                   nullptr, nullptr);
    return sigma_impl<double>(T, (const double *)C, (double *)S, (double *)CT, (double *)ST, epart, st,
                              (double2 *)zout, zipped);
}

hipError_t launch_pool(int vtype, const void *psi, const void *lam, const PairOp *ops, const uint32_t *lists,
                       int n_ops, int gx, int64_t nsa, int64_t nsb, double *partial, hipStream_t st) {
    const dim3 grid((unsigned)gx, (unsigned)n_ops), block(256);
    if (vtype == V_F64)
        hipLaunchKernelGGL(k_pool<double>, grid, block, 0, st, (const double *)psi, (const double *)lam, ops, lists,
                           nsa, nsb, partial);
    else if (vtype == V_F32)
        hipLaunchKernelGGL(k_pool<float>, grid, block, 0, st, (const float *)psi, (const float *)lam, ops, lists,
                           nsa, nsb, partial);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_string_h_values(double *val, const double *v2, const int32_t *desc, const uint32_t *str,
                                  const double *ht, int M, int64_t n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_string_h_values, dim3(blocks_for(n, 256)), dim3(256), 0, st, val, v2, desc, str, ht, M, n);
    return hipGetLastError();
}

hipError_t launch_csr_dense(const int64_t *rowptr, const int32_t *col, const double *val, double *out, int64_t n,
                            hipStream_t st) {
    hipLaunchKernelGGL(k_csr_dense, dim3((unsigned)n), dim3(256), 0, st, rowptr, col, val, out, n);
    return hipGetLastError();
}

hipError_t launch_ctranspose(bool cplex, const void *in, void *out, int64_t rows, int64_t cols, hipStream_t st) {
    const dim3 grid((unsigned)((cols + 31) / 32), (unsigned)((rows + 31) / 32));
    if (cplex)
        hipLaunchKernelGGL(k_transpose<double2>, grid, dim3(32, 8), 0, st, (const double2 *)in, (double2 *)out, rows, cols);
    else
        hipLaunchKernelGGL(k_transpose<double>, grid, dim3(32, 8), 0, st, (const double *)in, (double *)out, rows, cols);
    return hipGetLastError();
}

hipError_t launch_scatter_real(int precision, void *lam, const double *S, const uint64_t *Xa,
                               const uint64_t *Xb, const uint32_t *sa, const uint32_t *PPb, int64_t nsa,
                               int64_t nsb, hipStream_t st) {
    const unsigned gx = blocks_for(nsb, 256) > 64 ? 64 : blocks_for(nsb, 256);
    const dim3 grid(gx, (unsigned)nsa);
    if (precision == 0)
        hipLaunchKernelGGL(k_scatter_real<double2>, grid, dim3(256), 0, st, (double2 *)lam, S, Xa, Xb, sa, PPb, nsb);
    else
        hipLaunchKernelGGL(k_scatter_real<float2>, grid, dim3(256), 0, st, (float2 *)lam, S, Xa, Xb, sa, PPb, nsb);
    return hipGetLastError();
}

}  // namespace fsv
