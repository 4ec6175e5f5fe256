// Batched evaluation: many independent instances (own qubit count, electrons,
// integrals and operators), each getting energy + adjoint gradient, from one
// captured HIP graph.
//
// Each instance lives on its (N_alpha, N_beta) sector only, stored compactly
// as C[Ia][Ib] in the alpha-string-first product basis (the JW basis of the
// blocked qubit ordering restricted to the sector).  In that basis an
// excitation factorises into an alpha part and a beta part:
// tau|Ia Ib> = sign0 * s_a * s_b |Ia' Ib'>, so its active pairs are the
// product of an alpha pair list and a beta pair list (or "all strings" when
// the operator has no alpha / beta part).  Angles and integrals are real, so
// every amplitude stays real: the arena holds one double per amplitude.
//
// H C is evaluated row by row (one alpha string Ia per task):
//   S[Ia][Ib] = e_core C[Ia][Ib] + sum_J Ha[Ia][J] C[J][Ib] + sum_J Hb[Ib][J] C[Ia][J]
//             + sum_{e in exc(Ia)} sum_{f in exc(Ib)} s_e s_f (pq_e|rs_f) C[Ja_e][Jb_f]
// with Ha, Hb the same-spin string Hamiltonians (Slater-Condon rules) and
// exc(I) the single-excitation lists E_pq|J> = s |I>.  The task stages its own
// row, the rows C[Ja_e][:] and the weights s_e (pq_e|rs) in LDS, so the
// alpha-beta double sum reads LDS only.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/fsv.h"
#include "fsv_device.h"
#include "fsv_internal.h"

using namespace fsv;

namespace {

struct BInst {
    int32_t M, nsa, nsb, nexcA, nexcB, K, ref;
    int32_t ec;   // alpha excitations staged per LDS pass (even); 0: global-memory sigma;
                  // -1: factorised alpha-beta term with the row's intermediate in LDS
    int32_t wB;   // width of the beta string Hamiltonian in ELL form
    int32_t R;    // exact pivoted-Cholesky rank of (pq|rs) used by the factorised form (0: direct)
    int64_t dim;
    int64_t off_state;  // first double of psi in the arena; lam follows psi
    int64_t off_ops;    // first BOp
    int64_t off_k;      // first angle / gradient slot
    int64_t off_g;      // first double of (pq|rs)
    int64_t off_ha;     // first row pointer of the alpha string Hamiltonian (CSR)
    int64_t off_hb;     // first entry of the beta string Hamiltonian (ELL, [slot][Ib])
    int64_t off_excA;   // alpha excitation lists, [Ia][e]
    int64_t off_excB;   // beta excitation lists transposed, [f][Ib]
    int64_t off_task;   // first sigma task (row) of this instance
    int64_t off_lt;     // factor table [pq][l] (M^2 x kBLr, zero beyond R)
    int64_t off_da;     // per alpha string, then per beta string: the factor rows of its
                        // diagonal excitations summed ((nsa + nsb) x kBLr)
    int32_t ndA, ndB;   // diagonal entries at the end of each alpha / beta excitation list
    int32_t ssd;        // 1: k_pss computes the same-spin part of S (dense, matrix cores)
    int64_t off_hd;     // dense alpha string Hamiltonian (nsa x nsa), then the beta one
                        // transposed (nsb x nsb), both row-major
    int64_t off_init;   // first entry of this instance's initial-state list
    int32_t n_init;     // its length (0: the reference determinant)
    int32_t pad_init;
    double ecore;
};

constexpr int kBLr = 8;       // factor columns of the factorised form (ranks <= 8)
constexpr int kBLrStride = 9;  // LDS row stride (doubles) of its staged factors and intermediate

// Flat device tables of all instances.
struct BTabs {
    const double *g;
    const int64_t *hptr;
    const int32_t *hcol;
    const double *hval;
    const int32_t *ellc;
    const double *ellv;
    const uint32_t *excA, *excBT;
    const double *lt;
    const double *ldiag;
};

using BOp = PairOp;

__device__ inline void pair_of(const BInst &I, const BOp &op, const uint32_t *__restrict__ lists,
                               uint32_t t, uint32_t nb, int64_t &src, int64_t &dst, bool &neg) {
    const uint32_t u = t / nb, v = t - u * nb;
    uint32_t ia = u, ia2 = u, ib = v, ib2 = v;
    bool n = op.sign0 < 0;
    if (op.nA >= 0) {
        const uint32_t e = lists[op.offA + u];
        ia = e & 0x7FFFu;
        ia2 = (e >> 15) & 0x7FFFu;
        n ^= (e >> 31) != 0;
    }
    if (op.nB >= 0) {
        const uint32_t e = lists[op.offB + v];
        ib = e & 0x7FFFu;
        ib2 = (e >> 15) & 0x7FFFu;
        n ^= (e >> 31) != 0;
    }
    src = (int64_t)ia * I.nsb + ib;
    dst = (int64_t)ia2 * I.nsb + ib2;
    neg = n;
}

__device__ inline uint32_t pairs_of(const BInst &I, const BOp &op) {
    return (uint32_t)(op.nA >= 0 ? op.nA : I.nsa) * (uint32_t)(op.nB >= 0 ? op.nB : I.nsb);
}

// Row Ia of S = H C; returns this thread's share of sum_Ib C[Ia][Ib] S[Ia][Ib].
// Called by every thread of the workgroup (it synchronises); lds holds at
// least 2 nsb + (nsb + M^2) ec doubles when ec > 0.  SS: k_pss has already
// written the same-spin part of S (instances with ssd set).
template <bool SS>
__device__ double sigma_row(const BInst &I, int Ia, const double *__restrict__ C, double *__restrict__ S,
                            const BTabs &T, double *lds) {
    constexpr bool ss = SS;
    const int nsb = I.nsb, bs = blockDim.x, tid = threadIdx.x;
    const int M2 = I.M * I.M;
    const double *crowg = C + (int64_t)Ia * nsb;
    const int64_t *pa = T.hptr + I.off_ha;
    const int64_t q0 = pa[Ia], q1 = pa[Ia + 1];
    const int32_t *elc = T.ellc + I.off_hb;
    const double *elv = T.ellv + I.off_hb;
    const uint32_t *exa = T.excA + I.off_excA + (int64_t)Ia * I.nexcA;
    const uint32_t *exb = T.excBT + I.off_excB;
    const double *g = T.g + I.off_g;
    double eacc = 0.0;
    if (I.ec == 0) {  // rows too long for LDS: everything from global memory
        for (int ib = tid; ib < nsb; ib += bs) {
            const double x0 = crowg[ib];
            double a = I.ecore * x0;
            if (ss) {
                a += S[(int64_t)Ia * nsb + ib];
            } else {
                for (int64_t q = q0; q < q1; ++q) a += T.hval[q] * C[(int64_t)T.hcol[q] * nsb + ib];
                for (int q = 0; q < I.wB; ++q)
                    a += elv[(int64_t)q * nsb + ib] * crowg[elc[(int64_t)q * nsb + ib]];
            }
            for (int e = 0; e < I.nexcA; ++e) {
                const uint32_t wa = exa[e];
                const double *crj = C + (int64_t)(wa & 0xFFFFu) * nsb;
                const double *gp = g + (int64_t)((wa >> 16) & 0x1FFu) * M2;
                double b = 0.0;
                for (int f = 0; f < I.nexcB; ++f) {
                    const uint32_t wb = exb[(int64_t)f * nsb + ib];
                    const double v = gp[(wb >> 16) & 0x1FFu] * crj[wb & 0xFFFFu];
                    b += (wb >> 31) ? -v : v;
                }
                a += (wa >> 31) ? -b : b;
            }
            S[(int64_t)Ia * nsb + ib] = a;
            eacc += x0 * a;
        }
        return eacc;
    }
    if (I.ec < 0) {
        // factorised: (pq|rs) = sum_l L_l[pq] L_l[rs]; Y[Jb][l] = sum_e s_e L_l[pq_e]
        // C[Ja_e][Jb] built in LDS, then S[Ib] += sum_f s_f sum_l L_l[rs_f] Y[Jb_f][l]
        double *crow = lds, *acc = lds + nsb, *yr = lds + 2 * nsb, *lt = yr + (int64_t)nsb * kBLrStride;
        const double *ltg = T.lt + I.off_lt;
        const double *dag = T.ldiag + I.off_da, *dbg = dag + (int64_t)I.nsa * kBLr;
        const int noffA = I.nexcA - I.ndA, noffB = I.nexcB - I.ndB;
        double *dal = lt + kBLr;  // Ia's summed diagonal factors, in the unused last column of lt's rows
        __syncthreads();  // earlier readers of lds are done
        for (int j = tid; j < nsb; j += bs) crow[j] = crowg[j];
        for (int t = tid; t < M2 * kBLr; t += bs) lt[(t / kBLr) * kBLrStride + t % kBLr] = ltg[t];
        if (tid < kBLr) dal[tid * kBLrStride] = dag[(int64_t)Ia * kBLr + tid];  // M2 >= kBLr rows (host)
        __syncthreads();
        // Each loop below takes its list words kB at a time, loads first, so
        // the dependent gathers of a batch are in flight together (the sums
        // keep their order).
        constexpr int kB = 4, kBA = 8;  // alpha rows: coalesced row loads with uniform list words
        for (int ib = tid; ib < nsb; ib += bs) {
            double a = I.ecore * crow[ib];
            if (ss) {
                acc[ib] = a + S[(int64_t)Ia * nsb + ib];
                continue;
            }
            int64_t q = q0;
            for (; q + kBA <= q1; q += kBA) {
                double x[kBA];
#pragma unroll
                for (int u = 0; u < kBA; ++u) x[u] = C[(int64_t)T.hcol[q + u] * nsb + ib];
#pragma unroll
                for (int u = 0; u < kBA; ++u) a += T.hval[q + u] * x[u];
            }
            for (; q < q1; ++q) a += T.hval[q] * C[(int64_t)T.hcol[q] * nsb + ib];
            int qb = 0;
            for (; qb + kB <= I.wB; qb += kB) {
                int32_t cidx[kB];
                double wv[kB];
#pragma unroll
                for (int u = 0; u < kB; ++u) {
                    cidx[u] = elc[(int64_t)(qb + u) * nsb + ib];
                    wv[u] = elv[(int64_t)(qb + u) * nsb + ib];
                }
#pragma unroll
                for (int u = 0; u < kB; ++u) a += wv[u] * crow[cidx[u]];
            }
            for (; qb < I.wB; ++qb) a += elv[(int64_t)qb * nsb + ib] * crow[elc[(int64_t)qb * nsb + ib]];
            acc[ib] = a;
        }
        // a string's diagonal excitations (the last of its list) all map it
        // to itself: one term with its summed factor row
        for (int jb = tid; jb < nsb; jb += bs) {
            double y[kBLr];
#pragma unroll
            for (int l = 0; l < kBLr; ++l) y[l] = dal[l * kBLrStride] * crow[jb];
            auto step = [&](uint32_t wa, double x) {
                const double xv = (wa >> 31) ? -x : x;
                const double *w = lt + ((wa >> 16) & 0x1FFu) * kBLrStride;
#pragma unroll
                for (int l = 0; l < kBLr; ++l) y[l] += w[l] * xv;
            };
            int e = 0;
            for (; e + kB <= noffA; e += kB) {
                double x[kB];
#pragma unroll
                for (int u = 0; u < kB; ++u) x[u] = C[(int64_t)(exa[e + u] & 0xFFFFu) * nsb + jb];
#pragma unroll
                for (int u = 0; u < kB; ++u) step(exa[e + u], x[u]);
            }
            for (; e < noffA; ++e) step(exa[e], C[(int64_t)(exa[e] & 0xFFFFu) * nsb + jb]);
            // the beta diagonal term of element jb needs only Y[jb]: added here,
            // by the thread that wrote acc[jb]
            double dt = 0.0;
#pragma unroll
            for (int l = 0; l < kBLr; ++l) {
                yr[(int64_t)jb * kBLrStride + l] = y[l];
                dt += dbg[(int64_t)jb * kBLr + l] * y[l];
            }
            acc[jb] += dt;
        }
        __syncthreads();
        for (int ib = tid; ib < nsb; ib += bs) {
            double s = 0.0;
            auto step = [&](uint32_t wb) {
                const double *w = lt + ((wb >> 16) & 0x1FFu) * kBLrStride;
                const double *y = yr + (int64_t)(wb & 0xFFFFu) * kBLrStride;
                double t = 0.0;
#pragma unroll
                for (int l = 0; l < kBLr; ++l) t += w[l] * y[l];
                s += (wb >> 31) ? -t : t;
            };
            int f = 0;
            for (; f + kB <= noffB; f += kB) {
                uint32_t wb[kB];
#pragma unroll
                for (int u = 0; u < kB; ++u) wb[u] = exb[(int64_t)(f + u) * nsb + ib];
#pragma unroll
                for (int u = 0; u < kB; ++u) step(wb[u]);
            }
            for (; f < noffB; ++f) step(exb[(int64_t)f * nsb + ib]);
            const double a = acc[ib] + s;
            S[(int64_t)Ia * nsb + ib] = a;
            eacc += crow[ib] * a;
        }
        return eacc;
    }
    const int ec = I.ec;
    double *crow = lds, *acc = lds + nsb, *Rt = lds + 2 * nsb, *Wt = Rt + (int64_t)nsb * ec;
    __syncthreads();  // earlier readers of lds are done
    for (int j = tid; j < nsb; j += bs) crow[j] = crowg[j];
    __syncthreads();
    for (int ib = tid; ib < nsb; ib += bs) {
        double a = I.ecore * crow[ib];
        if (ss) {
            a += S[(int64_t)Ia * nsb + ib];
        } else {
            for (int64_t q = q0; q < q1; ++q) a += T.hval[q] * C[(int64_t)T.hcol[q] * nsb + ib];
            for (int q = 0; q < I.wB; ++q) a += elv[(int64_t)q * nsb + ib] * crow[elc[(int64_t)q * nsb + ib]];
        }
        acc[ib] = a;
    }
    for (int e0 = 0; e0 < I.nexcA; e0 += ec) {
        const int ne = min(ec, I.nexcA - e0), nep = (ne + 1) & ~1;
        __syncthreads();  // readers of the previous chunk are done
        // Rt[Jb][e] = C[Ja_e][Jb] and Wt[rs][e] = s_e (pq_e|rs); an odd chunk is
        // padded with a zero column so the dot products run over pairs
        for (int t = tid; t < nep * nsb; t += bs) {
            const int e = t / nsb, jb = t - e * nsb;
            double v = 0.0;
            if (e < ne) v = C[(int64_t)(exa[e0 + e] & 0xFFFFu) * nsb + jb];
            Rt[jb * ec + e] = v;
        }
        for (int t = tid; t < nep * M2; t += bs) {
            const int e = t / M2, rs = t - e * M2;
            double v = 0.0;
            if (e < ne) {
                const uint32_t wa = exa[e0 + e];
                v = g[(int64_t)((wa >> 16) & 0x1FFu) * M2 + rs];
                if (wa >> 31) v = -v;
            }
            Wt[rs * ec + e] = v;
        }
        __syncthreads();
        for (int ib = tid; ib < nsb; ib += bs) {
            double s = 0.0;
            for (int f = 0; f < I.nexcB; ++f) {
                const uint32_t wb = exb[(int64_t)f * nsb + ib];
                const double2 *r = (const double2 *)(Rt + (wb & 0xFFFFu) * ec);
                const double2 *w = (const double2 *)(Wt + ((wb >> 16) & 0x1FFu) * ec);
                double d = 0.0;
                for (int e = 0; e < nep / 2; ++e) {
                    const double2 x = r[e], y = w[e];
                    d += x.x * y.x + x.y * y.y;
                }
                s += (wb >> 31) ? -d : d;
            }
            acc[ib] += s;
        }
    }
    for (int ib = tid; ib < nsb; ib += bs) {  // same thread-to-column map as above
        S[(int64_t)Ia * nsb + ib] = acc[ib];
        eacc += crow[ib] * acc[ib];
    }
    return eacc;
}

// ---------------------------------------------------- persistent mode ----
// Workgroups take whole instances from a device counter (largest first) and
// run forward sweep, H C and the reverse adjoint sweep with workgroup
// barriers between operators.
__global__ __launch_bounds__(1024) void k_batch(
    const BInst *__restrict__ inst, const int *__restrict__ order, int count, int *counter,
    const BOp *__restrict__ ops, const uint32_t *__restrict__ lists, const double *__restrict__ cs,
    BTabs T, double *__restrict__ arena, double *__restrict__ grad, double *__restrict__ eout,
    const int64_t *__restrict__ init_idx, const double *__restrict__ init_val) {
    extern __shared__ double lds[];
    __shared__ int s_idx;
    for (;;) {
        if (threadIdx.x == 0) s_idx = atomicAdd(counter, 1);
        __syncthreads();
        const int idx = s_idx;
        __syncthreads();
        if (idx >= count) break;  // every wave of the workgroup leaves here
        const BInst I = inst[order[idx]];
        double *psi = arena + I.off_state;
        double *lam = psi + I.dim;

        for (int64_t t = threadIdx.x; t < I.dim; t += blockDim.x) psi[t] = (I.n_init == 0 && t == I.ref) ? 1.0 : 0.0;
        __syncthreads();
        for (int t = threadIdx.x; t < I.n_init; t += blockDim.x) psi[init_idx[I.off_init + t]] = init_val[I.off_init + t];
        __syncthreads();

        for (int k = 0; k < I.K; ++k) {  // forward sweep
            const BOp op = ops[I.off_ops + k];
            const double c = cs[2 * (I.off_k + k)], s = cs[2 * (I.off_k + k) + 1];
            const uint32_t np = pairs_of(I, op), nb = op.nB >= 0 ? op.nB : I.nsb;
            for (uint32_t t = threadIdx.x; t < np; t += blockDim.x) {
                int64_t xs, xd;
                bool neg;
                pair_of(I, op, lists, t, nb, xs, xd, neg);
                const double sg = neg ? -s : s;
                const double a = psi[xs], b = psi[xd];
                psi[xs] = c * a - sg * b;
                psi[xd] = c * b + sg * a;
            }
            __syncthreads();
        }

        double eacc = 0.0;  // lam = H psi, E = <psi|lam>
        for (int Ia = 0; Ia < I.nsa; ++Ia) eacc += sigma_row<false>(I, Ia, psi, lam, T, lds);
        const double E = block_sum(eacc);  // also orders lam before the sweep

        for (int k = I.K - 1; k >= 0; --k) {  // reverse adjoint sweep
            const BOp op = ops[I.off_ops + k];
            const double c = cs[2 * (I.off_k + k)], s = cs[2 * (I.off_k + k) + 1];
            const uint32_t np = pairs_of(I, op), nb = op.nB >= 0 ? op.nB : I.nsb;
            double acc = 0.0;
            for (uint32_t t = threadIdx.x; t < np; t += blockDim.x) {
                int64_t xs, xd;
                bool neg;
                pair_of(I, op, lists, t, nb, xs, xd, neg);
                const double a = psi[xs], b = psi[xd], la = lam[xs], lb = lam[xd];
                const double o = lb * a - la * b;
                acc += neg ? -o : o;
                const double sg = neg ? -s : s;
                psi[xs] = c * a + sg * b;
                psi[xd] = c * b - sg * a;
                lam[xs] = c * la + sg * lb;
                lam[xd] = c * lb - sg * la;
            }
            const double gk = block_sum(acc);  // also orders this op before the next
            if (threadIdx.x == 0) grad[I.off_k + k] = 2.0 * gk;
        }
        if (threadIdx.x == 0) eout[order[idx]] = E;
        __syncthreads();
    }
}

// ------------------------------------------------------- phased mode ----
// One launch per phase and operator index across all instances: workgroup
// (x, y) of a rotation launch serves instance y, slice x of gridDim.x; the
// H C launch has one workgroup per (instance, alpha string).  Kernel
// boundaries order the phases; no workgroup ever waits on another.

__global__ __launch_bounds__(256) void k_pinit(const BInst *__restrict__ inst, double *__restrict__ arena) {
    const BInst I = inst[blockIdx.y];
    double *psi = arena + I.off_state;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < I.dim;
         t += (int64_t)gridDim.x * blockDim.x)
        psi[t] = (I.n_init == 0 && t == I.ref) ? 1.0 : 0.0;
}

// Multi-determinant starts: workgroup y writes instance y's list (after
// k_pinit has cleared its state).
__global__ __launch_bounds__(64) void k_pinit_list(const BInst *__restrict__ inst, const int64_t *__restrict__ idx,
                                                   const double *__restrict__ val, double *__restrict__ arena) {
    const BInst I = inst[blockIdx.y];
    double *psi = arena + I.off_state;
    for (int t = threadIdx.x; t < I.n_init; t += blockDim.x) psi[idx[I.off_init + t]] = val[I.off_init + t];
}

__global__ __launch_bounds__(256) void k_pfwd(const BInst *__restrict__ inst, const BOp *__restrict__ ops,
                                              const uint32_t *__restrict__ lists,
                                              const double *__restrict__ cs, double *__restrict__ arena,
                                              int k) {
    const BInst I = inst[blockIdx.y];
    if (k >= I.K) return;
    const BOp op = ops[I.off_ops + k];
    const double c = cs[2 * (I.off_k + k)], s = cs[2 * (I.off_k + k) + 1];
    double *psi = arena + I.off_state;
    const uint32_t np = pairs_of(I, op), nb = op.nB >= 0 ? op.nB : I.nsb;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < np; t += gridDim.x * blockDim.x) {
        int64_t xs, xd;
        bool neg;
        pair_of(I, op, lists, t, nb, xs, xd, neg);
        const double sg = neg ? -s : s;
        const double a = psi[xs], b = psi[xd];
        psi[xs] = c * a - sg * b;
        psi[xd] = c * b + sg * a;
    }
}

typedef double dbl4 __attribute__((ext_vector_type(4)));

// Same-spin part of S = H C for instances with ssd set, on the FP64 matrix
// cores: S = Ha C + C Hb^T (Ha, Hb^T dense row-major, nsa x nsa and nsb x nsb;
// C, S row-major nsa x nsb in the arena).  One wavefront per 32 x 32 tile
// (task = instance, first row, first column), as 2 x 2 blocks of the 16 x 16
// x 4 FP64 MFMA: lane l feeds A[l % 16][l / 16] and B[l / 16][l % 16] of each
// step and holds D[4 r + l / 16][l % 16] in its result element r < 4 (checked
// on the device lane by lane).  Operands
// outside the matrices are read as zero (masked loads), and only the tile's
// entries inside S are written.
constexpr int kPssTile = 32;
constexpr int kPssK = 8;  // k steps per round: all their loads in flight before the MFMAs

__global__ __launch_bounds__(kWave) void k_pss(const BInst *__restrict__ inst, const int32_t *__restrict__ tasks,
                                               const double *__restrict__ hd, double *__restrict__ arena) {
    const int32_t *t = tasks + 3 * (int64_t)blockIdx.x;
    const BInst &I = inst[t[0]];
    const int m0 = t[1], n0 = t[2];
    const int nsa = I.nsa, nsb = I.nsb;
    const double *C = arena + I.off_state;
    double *S = arena + I.off_state + I.dim;
    const double *Ha = hd + I.off_hd, *Hbt = Ha + (int64_t)nsa * nsa;
    const int l = threadIdx.x, li = l & 15, lk = l >> 4;
    dbl4 acc[2][2];
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = dbl4{0.0, 0.0, 0.0, 0.0};
    // two products over their own inner dimension: (A, lda, B, ldb, K)
#pragma unroll
    for (int part = 0; part < 2; ++part) {
        const double *A = part == 0 ? Ha : C;
        const double *B = part == 0 ? C : Hbt;
        const int K = part == 0 ? nsa : nsb, lda = K;
        for (int k0 = 0; k0 < K; k0 += 4 * kPssK) {
            double a[kPssK][2], b[kPssK][2];
#pragma unroll
            for (int u = 0; u < kPssK; ++u) {
                const int kk = k0 + 4 * u + lk;
#pragma unroll
                for (int bi = 0; bi < 2; ++bi) {
                    const int m = m0 + 16 * bi + li;
                    a[u][bi] = (m < nsa && kk < K) ? A[(int64_t)m * lda + kk] : 0.0;
                }
#pragma unroll
                for (int bj = 0; bj < 2; ++bj) {
                    const int n = n0 + 16 * bj + li;
                    b[u][bj] = (kk < K && n < nsb) ? B[(int64_t)kk * nsb + n] : 0.0;
                }
            }
#pragma unroll
            for (int u = 0; u < kPssK; ++u)
#pragma unroll
                for (int bi = 0; bi < 2; ++bi)
#pragma unroll
                    for (int bj = 0; bj < 2; ++bj)
                        acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[u][bi], b[u][bj], acc[bi][bj], 0, 0, 0);
        }
    }
#pragma unroll
    for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int m = m0 + 16 * bi + 4 * r + lk, n = n0 + 16 * bj + li;
                if (m < nsa && n < nsb) S[(int64_t)m * nsb + n] = acc[bi][bj][r];
            }
}

// Row tasks task0 + blockIdx.x.  SS: the launch covers only instances with
// ssd set, after k_pss (their same-spin part of S is in place).
template <bool SS>
__global__ __launch_bounds__(256) void k_psigma(const BInst *__restrict__ inst, const int32_t *__restrict__ tinst,
                                                BTabs T, double *__restrict__ arena,
                                                double *__restrict__ epart, int64_t task0) {
    extern __shared__ double lds[];
    const int64_t task = task0 + blockIdx.x;
    const BInst I = inst[tinst[task]];
    const double *psi = arena + I.off_state;
    double *lam = arena + I.off_state + I.dim;
    const double e = block_sum(sigma_row<SS>(I, (int)(task - I.off_task), psi, lam, T, lds));
    if (threadIdx.x == 0) epart[task] = e;
}

__global__ __launch_bounds__(256) void k_prev(const BInst *__restrict__ inst, const BOp *__restrict__ ops,
                                              const uint32_t *__restrict__ lists,
                                              const double *__restrict__ cs, double *__restrict__ arena,
                                              int k, double *__restrict__ gpart) {
    const BInst I = inst[blockIdx.y];
    if (k >= I.K) return;  // uniform across the workgroup
    const BOp op = ops[I.off_ops + k];
    const double c = cs[2 * (I.off_k + k)], s = cs[2 * (I.off_k + k) + 1];
    double *psi = arena + I.off_state;
    double *lam = psi + I.dim;
    const uint32_t np = pairs_of(I, op), nb = op.nB >= 0 ? op.nB : I.nsb;
    double acc = 0.0;
    for (uint32_t t = blockIdx.x * blockDim.x + threadIdx.x; t < np; t += gridDim.x * blockDim.x) {
        int64_t xs, xd;
        bool neg;
        pair_of(I, op, lists, t, nb, xs, xd, neg);
        const double a = psi[xs], b = psi[xd], la = lam[xs], lb = lam[xd];
        const double o = lb * a - la * b;
        acc += neg ? -o : o;
        const double sg = neg ? -s : s;
        psi[xs] = c * a + sg * b;
        psi[xd] = c * b - sg * a;
        lam[xs] = c * la + sg * lb;
        lam[xd] = c * lb - sg * la;
    }
    acc = block_sum(acc);
    if (threadIdx.x == 0) gpart[(I.off_k + k) * gridDim.x + blockIdx.x] = acc;
}

// Ordered per-instance sums of the partials: E over the instance's row tasks
// and 2 * the per-operator sums.
__global__ __launch_bounds__(64) void k_preduce(const BInst *__restrict__ inst, int gx,
                                                const double *__restrict__ epart,
                                                const double *__restrict__ gpart,
                                                double *__restrict__ grad, double *__restrict__ eout) {
    const int y = blockIdx.x;
    const BInst I = inst[y];
    if (threadIdx.x == 0) {
        double e = 0.0;
        for (int r = 0; r < I.nsa; ++r) e += epart[I.off_task + r];
        eout[y] = e;
    }
    for (int k = threadIdx.x; k < I.K; k += blockDim.x) {
        double s = 0.0;
        for (int x = 0; x < gx; ++x) s += gpart[(I.off_k + k) * gx + x];
        grad[I.off_k + k] = 2.0 * s;
    }
}

// The same sums for packet runs, one wavefront per item: items below total_k
// are operators (global index; its partials are its run's packets, count[kk]
// of them at gpart[kk * pstride + slot]), the rest instances (energies).
// Lanes take every 64th partial, then a butterfly: a fixed order.
__global__ __launch_bounds__(64) void k_preduce_pk(const BInst *__restrict__ inst, const int32_t *__restrict__ count,
                                                   int64_t total_k, int pstride, const double *__restrict__ epart,
                                                   const double *__restrict__ gpart, double *__restrict__ grad,
                                                   double *__restrict__ eout) {
    const int64_t t = blockIdx.x;
    const int l = threadIdx.x;
    double s = 0.0;
    if (t < total_k) {
        for (int x = l; x < count[t]; x += kWave) s += gpart[t * pstride + x];
        s = wave_sum(s);
        if (l == 0) grad[t] = 2.0 * s;
    } else {
        const BInst I = inst[t - total_k];
        for (int r = l; r < I.nsa; r += kWave) s += epart[I.off_task + r];
        s = wave_sum(s);
        if (l == 0) eout[t - total_k] = s;
    }
}

// cos and sin of every angle (the first step of each captured evaluation).
__global__ __launch_bounds__(256) void k_cossin(const double *__restrict__ theta, double *__restrict__ cs,
                                                int64_t n) {
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        double s, c;
        sincos(theta[k], &s, &c);
        cs[2 * k] = c;
        cs[2 * k + 1] = s;
    }
}

__global__ void k_zero_int(int *p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

template <typename T>
int dmalloc(std::vector<void *> &owned, size_t &total, T **out, size_t count) {
    void *p = nullptr;
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(FSV_ENOMEM, "hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    }
    owned.push_back(p);
    total += bytes;
    *out = (T *)p;
    return FSV_OK;
}

}  // namespace

struct fsv_batch {
    int count = 0;
    int64_t total_k = 0;
    int64_t ntasks = 0;  // sigma row tasks = sum of the alpha string counts
    int64_t ntasks_ss = 0;  // the first ntasks_ss of them belong to instances with ssd set
    std::vector<BInst> inst;
    std::vector<int> order;
    std::vector<void *> owned;
    size_t bytes = 0;
    hipStream_t user = nullptr, work = nullptr;
    hipEvent_t ev_in = nullptr;
    BInst *d_inst = nullptr;
    int *d_order = nullptr, *d_counter = nullptr;
    int32_t *d_tinst = nullptr;
    BOp *d_ops = nullptr;
    uint32_t *d_lists = nullptr, *d_excA = nullptr, *d_excBT = nullptr;
    double *d_cs = nullptr, *d_theta = nullptr, *d_g = nullptr, *d_hval = nullptr, *d_ellv = nullptr;
    double *d_grad = nullptr, *d_e = nullptr;
    int64_t *d_hptr = nullptr;
    int32_t *d_hcol = nullptr, *d_ellc = nullptr;
    double *d_arena = nullptr;  // the caller's arena of the current call (arena_bytes)
    size_t arena_bytes = 0;
    double *h_pin = nullptr;  // theta (total_k) | spare (total_k) | grad (total_k) | E (count)
    int block = 256, per_cu = 2, cus = 256;
    int mode = 1;       // 0 persistent work-queue kernel, 1 phased launches, 2 packet runs
    int gx = 32;        // phased mode: workgroups per instance per rotation launch
    size_t lds_budget = 65536;  // LDS bytes a sigma workgroup may stage
    size_t lds_max = 65536;     // largest dynamic LDS the sigma kernels accept
    size_t lds_bytes = 0;       // dynamic LDS of the sigma kernels (max over instances)
    bool force_global = false;  // sigma from global memory only (FSV_BATCH_SIGMA=global)
    int kmax = 0;
    double *d_epart = nullptr, *d_gpart = nullptr;
    size_t part_cap = 0;  // workgroups per instance the gradient partials hold
    // dense same-spin products (k_pss) of the instances with ssd set
    double *d_hd = nullptr;
    int32_t *d_pss = nullptr;  // tasks: instance, first row, first column
    int64_t n_pss = 0;
    bool use_graph = true;
    hipGraphExec_t graph = nullptr;
    // packet runs (mode 2): one launch per run index, the runs of all instances
    BatchPackets pk;
    bool pk_ok = false;
    uint32_t *d_pent = nullptr, *d_preg = nullptr;
    int32_t *d_pcount = nullptr;
    double *d_pgpart = nullptr;
    double *d_lt = nullptr, *d_ldiag = nullptr;
    // multi-determinant starts: per instance (qubits, alpha, beta electrons,
    // ordering) on the host, and the concatenated sector lists on the device
    std::vector<std::array<int32_t, 4>> shape;
    std::vector<std::vector<int64_t>> init_idx;
    std::vector<std::vector<double>> init_val;
    int64_t *d_init_idx = nullptr;
    double *d_init_val = nullptr;
    size_t init_bytes = 0;
    int64_t n_init_total = 0;
    BTabs tabs() const { return BTabs{d_g, d_hptr, d_hcol, d_hval, d_ellc, d_ellv, d_excA, d_excBT, d_lt, d_ldiag}; }
    ~fsv_batch() {
        if (work) (void)hipStreamSynchronize(work);
        if (graph) (void)hipGraphExecDestroy(graph);
        for (void *p : owned) (void)hipFree(p);
        if (d_init_idx) (void)hipFree(d_init_idx);
        if (d_init_val) (void)hipFree(d_init_val);
        if (h_pin) (void)hipHostFree(h_pin);
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (work) (void)hipStreamDestroy(work);
    }
};

namespace {

#define BHIP(expr)                                                                          \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(FSV_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));        \
    } while (0)

// Per-instance alpha-excitation chunk for an LDS budget (bytes): the largest
// even ec with 2 nsb + (nsb + M^2) ec doubles within the budget, capped at the
// whole list; 0 (global-memory sigma) when not even two fit.  Uploads the
// instance table.
int set_lds_budget(fsv_batch &B, size_t budget) {
    budget = std::min(budget, B.lds_max);
    size_t need = 0;
    for (BInst &I : B.inst) {
        const int64_t nsb = I.nsb, M2 = (int64_t)I.M * I.M;
        if (I.R > 0 && !B.force_global) {  // factorised form when its row fits
            const size_t nf = (size_t)8 * (2 * nsb + (nsb + M2) * kBLrStride);
            if (nf <= budget) {
                I.ec = -1;
                need = std::max(need, nf);
                continue;
            }
        }
        const int64_t room = (int64_t)(budget / 8) - 2 * nsb;
        int64_t ec = room > 0 ? (room / (nsb + M2)) & ~1LL : 0;
        ec = std::min<int64_t>(ec, (I.nexcA + 1) & ~1);
        if (B.force_global || ec < 2) ec = 0;
        I.ec = (int32_t)ec;
        if (ec) need = std::max(need, (size_t)(8 * (2 * nsb + (nsb + M2) * ec)));
    }
    B.lds_budget = budget;
    B.lds_bytes = need;
    BHIP(hipMemcpy(B.d_inst, B.inst.data(), sizeof(BInst) * B.inst.size(), hipMemcpyHostToDevice));
    return FSV_OK;
}

// H C of every instance: the dense same-spin products of the instances with
// ssd set, their rows, then the rows of the others.
hipError_t launch_sigma(fsv_batch &B, const BTabs &T) {
    if (B.n_pss > 0) {
        hipLaunchKernelGGL(k_pss, dim3((unsigned)B.n_pss), dim3(kWave), 0, B.work, B.d_inst, B.d_pss, B.d_hd,
                           B.d_arena);
        hipLaunchKernelGGL(k_psigma<true>, dim3((unsigned)B.ntasks_ss), dim3(256), B.lds_bytes, B.work, B.d_inst,
                           B.d_tinst, T, B.d_arena, B.d_epart, (int64_t)0);
    }
    const int64_t rest = B.ntasks - (B.n_pss > 0 ? B.ntasks_ss : 0);
    if (rest > 0)
        hipLaunchKernelGGL(k_psigma<false>, dim3((unsigned)rest), dim3(256), B.lds_bytes, B.work, B.d_inst,
                           B.d_tinst, T, B.d_arena, B.d_epart, B.ntasks - rest);
    return hipGetLastError();
}

hipError_t launch_init_lists(fsv_batch &B) {
    if (B.n_init_total == 0) return hipSuccess;
    hipLaunchKernelGGL(k_pinit_list, dim3(1, (unsigned)B.count), dim3(64), 0, B.work, B.d_inst, B.d_init_idx,
                       B.d_init_val, B.d_arena);
    return hipGetLastError();
}

int enqueue(fsv_batch &B) {
    const BTabs T = B.tabs();
    if (B.total_k) {
        hipLaunchKernelGGL(k_cossin, dim3(blocks_for(B.total_k, 256)), dim3(256), 0, B.work, B.d_theta, B.d_cs,
                           B.total_k);
        BHIP(hipGetLastError());
    }
    if (B.mode == 2) {
        hipLaunchKernelGGL(k_pinit, dim3((unsigned)B.gx, (unsigned)B.count), dim3(256), 0, B.work, B.d_inst,
                           B.d_arena);
        BHIP(hipGetLastError());
        BHIP(launch_init_lists(B));
        const BatchPackets &P = B.pk;
        for (int r = 0; r < P.runs; ++r)
            BHIP(launch_batch_packets(false, B.d_arena, B.d_pent + P.ent_off[r], B.d_preg + P.reg_off[r], P.wr[r],
                                      P.npk[r], B.d_cs, nullptr, P.pstride, B.work));
        BHIP(launch_sigma(B, T));
        for (int r = P.runs - 1; r >= 0; --r)
            BHIP(launch_batch_packets(true, B.d_arena, B.d_pent + P.ent_off[r], B.d_preg + P.reg_off[r], P.wr[r],
                                      P.npk[r], B.d_cs, B.d_pgpart, P.pstride, B.work));
        hipLaunchKernelGGL(k_preduce_pk, dim3((unsigned)(B.total_k + B.count)), dim3(kWave), 0, B.work, B.d_inst,
                           B.d_pcount, B.total_k, P.pstride, B.d_epart, B.d_pgpart, B.d_grad, B.d_e);
        BHIP(hipGetLastError());
        return FSV_OK;
    }
    if (B.mode == 1) {
        const dim3 grid((unsigned)B.gx, (unsigned)B.count);
        hipLaunchKernelGGL(k_pinit, grid, dim3(256), 0, B.work, B.d_inst, B.d_arena);
        BHIP(hipGetLastError());
        BHIP(launch_init_lists(B));
        for (int k = 0; k < B.kmax; ++k) {
            hipLaunchKernelGGL(k_pfwd, grid, dim3(256), 0, B.work, B.d_inst, B.d_ops, B.d_lists, B.d_cs,
                               B.d_arena, k);
            BHIP(hipGetLastError());
        }
        BHIP(launch_sigma(B, T));
        for (int k = B.kmax - 1; k >= 0; --k) {
            hipLaunchKernelGGL(k_prev, grid, dim3(256), 0, B.work, B.d_inst, B.d_ops, B.d_lists, B.d_cs,
                               B.d_arena, k, B.d_gpart);
            BHIP(hipGetLastError());
        }
        hipLaunchKernelGGL(k_preduce, dim3((unsigned)B.count), dim3(64), 0, B.work, B.d_inst, B.gx,
                           B.d_epart, B.d_gpart, B.d_grad, B.d_e);
        BHIP(hipGetLastError());
        return FSV_OK;
    }
    hipLaunchKernelGGL(k_zero_int, dim3(1), dim3(64), 0, B.work, B.d_counter);
    BHIP(hipGetLastError());
    const int grid = std::max(1, std::min(B.count, B.cus * B.per_cu));
    hipLaunchKernelGGL(k_batch, dim3(grid), dim3(B.block), B.lds_bytes, B.work, B.d_inst, B.d_order,
                       B.count, B.d_counter, B.d_ops, B.d_lists, B.d_cs, T, B.d_arena, B.d_grad, B.d_e,
                       (const int64_t *)B.d_init_idx, (const double *)B.d_init_val);
    BHIP(hipGetLastError());
    return FSV_OK;
}

int launch(fsv_batch &B) {
    if (!B.use_graph) return enqueue(B);
    if (!B.graph) {
        BHIP(hipStreamBeginCapture(B.work, hipStreamCaptureModeThreadLocal));
        int rc = enqueue(B);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(B.work, &g);
        if (rc) {
            if (g) (void)hipGraphDestroy(g);
            return rc;
        }
        if (e != hipSuccess) return fail(FSV_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
        e = hipGraphInstantiate(&B.graph, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e != hipSuccess) {
            B.graph = nullptr;
            return fail(FSV_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
        }
    }
    BHIP(hipGraphLaunch(B.graph, B.work));
    return FSV_OK;
}

int run(fsv_batch &B, const double *theta, double *E_out, double *grad_out) {
    double *th = B.h_pin;
    for (int64_t k = 0; k < B.total_k; ++k) {
        if (!std::isfinite(theta[k])) return fail(FSV_ENONFINITE, "non-finite theta at %lld", (long long)k);
        th[k] = theta[k];
    }
    if (!stream_idle(B.user)) {  // an idle caller's stream has nothing to order against
        BHIP(hipEventRecord(B.ev_in, B.user));
        BHIP(hipStreamWaitEvent(B.work, B.ev_in, 0));
    }
    if (B.total_k)
        BHIP(hipMemcpyAsync(B.d_theta, th, sizeof(double) * B.total_k, hipMemcpyHostToDevice, B.work));
    int rc = launch(B);
    if (rc) return rc;
    double *hg = B.h_pin + 2 * B.total_k, *he = hg + B.total_k;
    if (B.total_k)
        BHIP(hipMemcpyAsync(hg, B.d_grad, sizeof(double) * B.total_k, hipMemcpyDeviceToHost, B.work));
    BHIP(hipMemcpyAsync(he, B.d_e, sizeof(double) * B.count, hipMemcpyDeviceToHost, B.work));
    BHIP(hipStreamSynchronize(B.work));  // the batch's work is complete: later work on the caller's stream follows it
    if (E_out) std::memcpy(E_out, he, sizeof(double) * B.count);
    if (grad_out && B.total_k) std::memcpy(grad_out, hg, sizeof(double) * B.total_k);
    return FSV_OK;
}

}  // namespace

extern "C" {

int fsv_batch_create(fsv_batch **out, const fsv_problem *problems, int32_t count, void *hip_stream) {
    if (!out) return fail(FSV_EINVAL, "out is NULL");
    *out = nullptr;
    if (!problems || count <= 0) return fail(FSV_EINVAL, "need at least one problem");
    for (int i = 0; i < count; ++i) {
        int rc = validate_problem(&problems[i]);
        if (rc) return fail(rc, "instance %d: %s", i, fsv_last_error());
        if (problems[i].precision != 0)
            return fail(FSV_EINVAL, "instance %d: batches compute in FP64 (precision 0)", i);
        if (problems[i].n_qubits > 24)
            return fail(FSV_EINVAL, "instance %d: batches take at most 24 qubits (use a plan)", i);
    }
    fsv_batch *B = new (std::nothrow) fsv_batch();
    if (!B) return fail(FSV_ENOMEM, "batch allocation failed");
    B->count = count;
    B->user = (hipStream_t)hip_stream;
    B->use_graph = std::getenv("FSV_NO_GRAPH") == nullptr;
    int env_mode = -1;
    if (const char *m = std::getenv("FSV_BATCH_MODE"))
        env_mode = std::strcmp(m, "persistent") == 0 ? 0 : (std::strcmp(m, "packets") == 0 ? 2 : 1);
    bool lr_off = false;
    // same-spin products: dense on the matrix cores (default) or sparse rows
    // (FSV_BATCH_SAME_SPIN=sparse)
    const char *ssm = std::getenv("FSV_BATCH_SAME_SPIN");
    const bool ss_sparse = ssm && std::strcmp(ssm, "sparse") == 0;
    if (const char *m = std::getenv("FSV_BATCH_SIGMA")) {
        B->force_global = std::strcmp(m, "global") == 0;
        lr_off = std::strcmp(m, "direct") == 0;
    }

    std::vector<BOp> ops;
    std::vector<uint32_t> lists, excA, excBT;
    std::vector<double> gall, hval, ellv, ltall, ldiag, hdense;
    std::vector<int32_t> pss;
    std::vector<int64_t> hptr;
    std::vector<int32_t> hcol, ellc;
    std::vector<double> cost(count);
    int64_t state = 0, kk = 0;
    for (int i = 0; i < count; ++i) {
        const fsv_problem &p = problems[i];
        const int M = p.n_qubits / 2;
        BInst I{};
        I.M = M;
        I.K = p.n_ops;
        std::vector<uint32_t> sa = strings_of(M, p.n_alpha), sb = strings_of(M, p.n_beta);
        std::vector<int32_t> ra(1u << M, -1), rb(1u << M, -1);
        for (size_t t = 0; t < sa.size(); ++t) ra[sa[t]] = (int32_t)t;
        for (size_t t = 0; t < sb.size(); ++t) rb[sb[t]] = (int32_t)t;
        I.nsa = (int32_t)sa.size();
        I.nsb = (int32_t)sb.size();
        I.dim = (int64_t)I.nsa * I.nsb;
        I.ref = 0;  // both reference strings are the first (lowest) masks
        I.off_state = state;
        state += 2 * I.dim;
        I.off_ops = (int64_t)ops.size();
        I.off_k = kk;
        kk += p.n_ops;
        I.ecore = p.e_core;
        I.off_g = (int64_t)gall.size();
        gall.insert(gall.end(), p.g, p.g + (size_t)M * M * M * M);
        // alpha string Hamiltonian as CSR (row pointers index hcol / hval globally)
        std::vector<int64_t> ptr;
        std::vector<int32_t> col;
        std::vector<double> val;
        build_string_h(M, sa, ra, p.h, p.g, ptr, col, val);
        const int64_t base = (int64_t)hcol.size();
        I.off_ha = (int64_t)hptr.size();
        for (int64_t v : ptr) hptr.push_back(v + base);
        hcol.insert(hcol.end(), col.begin(), col.end());
        hval.insert(hval.end(), val.begin(), val.end());
        const double nnz_a = (double)col.size() / std::max(1, I.nsa);
        // dense copies for the matrix-core same-spin product, on instances
        // with at least one full 16 x 16 block each way
        I.ssd = !ss_sparse && I.nsa >= 16 && I.nsb >= 16;
        I.off_hd = (int64_t)hdense.size();
        if (I.ssd) {
            hdense.resize(hdense.size() + (size_t)I.nsa * I.nsa + (size_t)I.nsb * I.nsb, 0.0);
            for (int r = 0; r < I.nsa; ++r)
                for (int64_t q = ptr[r]; q < ptr[r + 1]; ++q) hdense[(size_t)(I.off_hd + (int64_t)r * I.nsa + col[q])] = val[q];
        }
        // beta string Hamiltonian as transposed ELL: slot q of row Ib at [q][Ib],
        // padded with zero weights on the diagonal
        build_string_h(M, sb, rb, p.h, p.g, ptr, col, val);
        if (I.ssd) {  // Hb transposed: Hbt[Jb][Ib] = Hb[Ib][Jb]
            const int64_t o = I.off_hd + (int64_t)I.nsa * I.nsa;
            for (int r = 0; r < I.nsb; ++r)
                for (int64_t q = ptr[r]; q < ptr[r + 1]; ++q) hdense[(size_t)(o + (int64_t)col[q] * I.nsb + r)] = val[q];
            for (int m0 = 0; m0 < I.nsa; m0 += kPssTile)
                for (int n0 = 0; n0 < I.nsb; n0 += kPssTile) pss.insert(pss.end(), {i, m0, n0});
        }
        int w = 0;
        for (int r = 0; r < I.nsb; ++r) w = std::max<int>(w, (int)(ptr[r + 1] - ptr[r]));
        I.wB = w;
        I.off_hb = (int64_t)ellc.size();
        ellc.resize(ellc.size() + (size_t)w * I.nsb);
        ellv.resize(ellv.size() + (size_t)w * I.nsb, 0.0);
        for (int r = 0; r < I.nsb; ++r)
            for (int q = 0; q < w; ++q) {
                const int64_t at = I.off_hb + (int64_t)q * I.nsb + r, src = ptr[r] + q;
                const bool real = src < ptr[r + 1];
                ellc[at] = real ? col[src] : r;
                ellv[at] = real ? val[src] : 0.0;
            }
        std::vector<uint32_t> ea, eb;
        build_exc(M, sa, ra, ea, I.nexcA);
        build_exc(M, sb, rb, eb, I.nexcB);
        I.off_excA = (int64_t)excA.size();
        excA.insert(excA.end(), ea.begin(), ea.end());
        I.off_excB = (int64_t)excBT.size();
        excBT.resize(excBT.size() + (size_t)I.nexcB * I.nsb);
        for (int r = 0; r < I.nsb; ++r)
            for (int f = 0; f < I.nexcB; ++f)
                excBT[I.off_excB + (int64_t)f * I.nsb + r] = eb[(size_t)r * I.nexcB + f];
        // exact low-rank factors of (pq|rs) for the factorised alpha-beta term,
        // accepted as for a plan: rank <= 8, fewer multiply-adds, and g
        // reproduced to 1e-12 relative
        I.R = 0;
        I.off_lt = (int64_t)ltall.size();
        I.off_da = (int64_t)ldiag.size();
        I.ndA = __builtin_popcount(sa[0]);
        I.ndB = __builtin_popcount(sb[0]);
        if (!lr_off && I.nexcA > 0 && I.nexcB > 0 && M * M >= kBLr) {  // (the kernel keeps 8 values in lt's rows)
            const int M2 = M * M;
            std::vector<double> L;
            const int R = pivoted_cholesky(M2, p.g, 1e-14, L);
            if (R > 0 && R <= kBLr && (int64_t)R * (I.nexcA + I.nexcB) < (int64_t)I.nexcA * I.nexcB) {
                double gmax = 0.0, err = 0.0;
                for (int a = 0; a < M2; ++a)
                    for (int b = 0; b < M2; ++b) {
                        double v = 0.0;
                        for (int k = 0; k < R; ++k) v += L[(size_t)k * M2 + a] * L[(size_t)k * M2 + b];
                        gmax = std::max(gmax, std::fabs(p.g[(size_t)a * M2 + b]));
                        err = std::max(err, std::fabs(v - p.g[(size_t)a * M2 + b]));
                    }
                if (err <= 1e-12 * std::max(1.0, gmax)) {
                    I.R = R;
                    ltall.resize(ltall.size() + (size_t)M2 * kBLr, 0.0);
                    for (int k = 0; k < R; ++k)
                        for (int a = 0; a < M2; ++a) ltall[(size_t)I.off_lt + (size_t)a * kBLr + k] = L[(size_t)k * M2 + a];
                    const std::vector<double> lt(ltall.begin() + I.off_lt, ltall.end());
                    const std::vector<double> da = diag_factor_sums(M, sa, lt, kBLr), db = diag_factor_sums(M, sb, lt, kBLr);
                    ldiag.insert(ldiag.end(), da.begin(), da.end());
                    ldiag.insert(ldiag.end(), db.begin(), db.end());
                }
            }
        }
        // operators in the alpha-first basis = the blocked JW ordering (qubit
        // excitations carry the signs of the instance's own qubit ordering)
        double pairs = 0.0;
        for (int k = 0; k < p.n_ops; ++k) {
            const BOp o = p.excitation ? build_pair_op_qeb(M, p.ordering, p.ops + 4 * k, sa, ra, sb, rb, lists)
                                       : build_pair_op(M, p.ops + 4 * k, sa, ra, sb, rb, lists);
            pairs += (double)(o.nA >= 0 ? o.nA : I.nsa) * (double)(o.nB >= 0 ? o.nB : I.nsb);
            ops.push_back(o);
        }
        cost[i] = (double)I.dim * (nnz_a + w + (I.R ? 2.0 * I.R * (I.nexcA + I.nexcB) : (double)I.nexcA * I.nexcB)) +
                  3.0 * pairs;
        // bounds of this instance's tables as the batch kernels read them
        {
            bool good = I.nsa <= 32768 && I.nsb <= 32768 && M * M <= 511;
            for (int k = 0; good && k < p.n_ops; ++k) {
                const BOp &o = ops[(size_t)I.off_ops + k];
                for (int side = 0; side < 2 && good; ++side) {
                    const int32_t n = side ? o.nB : o.nA;
                    const int64_t off = side ? o.offB : o.offA, ns = side ? I.nsb : I.nsa;
                    if (n < -1 || (n >= 0 && off + n > (int64_t)lists.size())) good = false;
                    for (int32_t u = 0; good && u < n; ++u) {
                        const uint32_t e = lists[off + u];
                        good = (int64_t)(e & 0x7FFFu) < ns && (int64_t)((e >> 15) & 0x7FFFu) < ns;
                    }
                }
            }
            auto exc_ok = [&](const std::vector<uint32_t> &ex, int nexc, int ns, int nd) {
                if ((int64_t)ex.size() != (int64_t)ns * nexc || nd > nexc) return false;
                for (int r = 0; r < ns; ++r)
                    for (int e = 0; e < nexc; ++e) {
                        const uint32_t x = ex[(size_t)r * nexc + e];
                        if ((int)(x & 0xFFFFu) >= ns || (int)((x >> 16) & 0x1FFu) >= M * M) return false;
                        if (e >= nexc - nd && (x & 0xFFFFu) != (uint32_t)r) return false;
                    }
                return true;
            };
            good = good && exc_ok(ea, I.nexcA, I.nsa, I.ndA) && exc_ok(eb, I.nexcB, I.nsb, I.ndB);
            for (int64_t r = 0; good && r < I.nsa; ++r)
                for (int64_t q = hptr[I.off_ha + r] - base; good && q < hptr[I.off_ha + r + 1] - base; ++q)
                    good = hcol[base + q] >= 0 && hcol[base + q] < I.nsa;
            for (size_t q = 0; good && q < (size_t)w * I.nsb; ++q)
                good = ellc[I.off_hb + q] >= 0 && ellc[I.off_hb + q] < I.nsb;
            if (!good) {
                delete B;
                return fail(FSV_EINVAL, "internal: instance %d tables out of range", i);
            }
        }
        B->inst.push_back(I);
        B->shape.push_back({p.n_qubits, p.n_alpha, p.n_beta, p.ordering});
    }
    B->init_idx.assign(count, {});
    B->init_val.assign(count, {});
    B->total_k = kk;
    for (int i = 0; i < count; ++i) B->kmax = std::max(B->kmax, problems[i].n_ops);
    B->part_cap = 64;
    B->order.resize(count);
    std::iota(B->order.begin(), B->order.end(), 0);
    std::stable_sort(B->order.begin(), B->order.end(), [&](int a, int b) { return cost[a] > cost[b]; });
    // sigma row tasks: the instances whose same-spin part comes from k_pss
    // first, then the others, most expensive first within each group; each
    // instance's rows are contiguous so its energy partials sum in a fixed order
    std::vector<int32_t> tinst;
    for (int pass = 0; pass < 2; ++pass) {
        for (int i : B->order) {
            if ((B->inst[i].ssd != 0) != (pass == 0)) continue;
            B->inst[i].off_task = (int64_t)tinst.size();
            tinst.insert(tinst.end(), (size_t)B->inst[i].nsa, i);
        }
        if (pass == 0) B->ntasks_ss = (int64_t)tinst.size();
    }
    B->ntasks = (int64_t)tinst.size();

    int rc = FSV_OK;
    auto fin = [&](int code) {
        if (code) delete B;
        return code;
    };
    hipDeviceProp_t prop;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
        delete B;
        return fail(FSV_EDEVICE, "no HIP device");
    }
    B->cus = prop.multiProcessorCount;
    if (hipStreamCreateWithFlags(&B->work, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming) != hipSuccess) {
        delete B;
        return fail(FSV_EDEVICE, "stream/event creation failed");
    }
    if (hipHostMalloc((void **)&B->h_pin, sizeof(double) * (3 * kk + count + 8), hipHostMallocDefault) != hipSuccess) {
        delete B;
        return fail(FSV_ENOMEM, "pinned host buffer");
    }
    // dynamic LDS limit of the sigma kernels: a CU's 160 KiB less their static
    // LDS, or the default 64 KiB if the attribute cannot be raised
    B->lds_max = 163840;
    for (const void *f : {(const void *)k_psigma<true>, (const void *)k_psigma<false>, (const void *)k_batch}) {
        hipFuncAttributes fa;
        size_t lim = 163840;
        if (hipFuncGetAttributes(&fa, f) == hipSuccess) lim -= fa.sharedSizeBytes;
        if (hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lim) != hipSuccess) {
            (void)hipGetLastError();
            lim = 65536 - (lim < 163840 ? 163840 - lim : 0);
        }
        B->lds_max = std::min(B->lds_max, lim);
    }
    auto& o = B->owned;
    if ((rc = dmalloc(o, B->bytes, &B->d_inst, B->inst.size())) || (rc = dmalloc(o, B->bytes, &B->d_order, count)) ||
        (rc = dmalloc(o, B->bytes, &B->d_counter, 4)) || (rc = dmalloc(o, B->bytes, &B->d_tinst, tinst.size())) ||
        (rc = dmalloc(o, B->bytes, &B->d_ops, ops.size())) || (rc = dmalloc(o, B->bytes, &B->d_lists, lists.size())) ||
        (rc = dmalloc(o, B->bytes, &B->d_excA, excA.size())) || (rc = dmalloc(o, B->bytes, &B->d_excBT, excBT.size())) ||
        (rc = dmalloc(o, B->bytes, &B->d_cs, 2 * (size_t)kk)) || (rc = dmalloc(o, B->bytes, &B->d_theta, std::max<size_t>(kk, 1))) ||
        (rc = dmalloc(o, B->bytes, &B->d_g, gall.size())) ||
        (rc = dmalloc(o, B->bytes, &B->d_hval, hval.size())) || (rc = dmalloc(o, B->bytes, &B->d_hptr, hptr.size())) ||
        (rc = dmalloc(o, B->bytes, &B->d_hcol, hcol.size())) || (rc = dmalloc(o, B->bytes, &B->d_ellc, ellc.size())) ||
        (rc = dmalloc(o, B->bytes, &B->d_ellv, ellv.size())) || (rc = dmalloc(o, B->bytes, &B->d_grad, (size_t)kk)) ||
        (rc = dmalloc(o, B->bytes, &B->d_e, (size_t)count)) ||
        (rc = dmalloc(o, B->bytes, &B->d_epart, (size_t)B->ntasks)) || (rc = dmalloc(o, B->bytes, &B->d_lt, std::max<size_t>(ltall.size(), 1))) ||
        (rc = dmalloc(o, B->bytes, &B->d_ldiag, std::max<size_t>(ldiag.size(), 1))) ||
        (rc = dmalloc(o, B->bytes, &B->d_hd, std::max<size_t>(hdense.size(), 1))) ||
        (rc = dmalloc(o, B->bytes, &B->d_pss, std::max<size_t>(pss.size(), 1))) ||
        (rc = dmalloc(o, B->bytes, &B->d_gpart, (size_t)kk * B->part_cap)))
        return fin(rc);
    B->arena_bytes = 8 * (size_t)std::max<int64_t>(state, 1);
    struct Up { void *d; const void *h; size_t n; };
    const Up ups[] = {
        {B->d_order, B->order.data(), sizeof(int) * count},
        {B->d_tinst, tinst.data(), 4 * tinst.size()},
        {B->d_ops, ops.data(), sizeof(BOp) * ops.size()},
        {B->d_lists, lists.data(), 4 * lists.size()},
        {B->d_excA, excA.data(), 4 * excA.size()},
        {B->d_excBT, excBT.data(), 4 * excBT.size()},
        {B->d_g, gall.data(), 8 * gall.size()},
        {B->d_hval, hval.data(), 8 * hval.size()},
        {B->d_hptr, hptr.data(), 8 * hptr.size()},
        {B->d_hcol, hcol.data(), 4 * hcol.size()},
        {B->d_ellc, ellc.data(), 4 * ellc.size()},
        {B->d_ellv, ellv.data(), 8 * ellv.size()},
        {B->d_lt, ltall.data(), 8 * ltall.size()},
        {B->d_ldiag, ldiag.data(), 8 * ldiag.size()},
        {B->d_hd, hdense.data(), 8 * hdense.size()},
        {B->d_pss, pss.data(), 4 * pss.size()},
    };
    B->n_pss = (int64_t)pss.size() / 3;
    for (const Up &u : ups)
        if (u.n && hipMemcpy(u.d, u.h, u.n, hipMemcpyHostToDevice) != hipSuccess)
            return fin(fail(FSV_EDEVICE, "upload failed"));
    if ((rc = set_lds_budget(*B, B->lds_budget))) return fin(rc);
    // packet runs, when every instance is small enough (the default mode then)
    bool small = true;
    for (const BInst &I : B->inst) small = small && I.dim <= packet_default_dim();
    if (small && kk > 0) {
        std::vector<BatchPacketInst> pi;
        for (const BInst &I : B->inst) pi.push_back({I.nsa, I.nsb, I.off_state, I.off_ops, I.off_k, I.K});
        if ((rc = build_batch_packets(pi, ops, lists, B->pk))) return fin(rc);
        const BatchPackets &P = B->pk;
        if ((rc = dmalloc(o, B->bytes, &B->d_pent, std::max<size_t>(P.ent.size(), 1))) ||
            (rc = dmalloc(o, B->bytes, &B->d_preg, std::max<size_t>(P.reg.size(), 1))) ||
            (rc = dmalloc(o, B->bytes, &B->d_pcount, (size_t)kk)) || (rc = dmalloc(o, B->bytes, &B->d_pgpart, (size_t)kk * P.pstride)))
            return fin(rc);
        if ((!P.ent.empty() && hipMemcpy(B->d_pent, P.ent.data(), 4 * P.ent.size(), hipMemcpyHostToDevice) != hipSuccess) ||
            (!P.reg.empty() && hipMemcpy(B->d_preg, P.reg.data(), 4 * P.reg.size(), hipMemcpyHostToDevice) != hipSuccess) ||
            hipMemcpy(B->d_pcount, P.count.data(), 4 * (size_t)kk, hipMemcpyHostToDevice) != hipSuccess)
            return fin(fail(FSV_EDEVICE, "upload of packet runs failed"));
        B->pk_ok = true;
        B->mode = 2;
    }
    if (env_mode >= 0) B->mode = env_mode == 2 && !B->pk_ok ? 1 : env_mode;
    *out = B;
    clear_error();
    return FSV_OK;
}

int fsv_batch_destroy(fsv_batch *B) {
    delete B;
    return FSV_OK;
}

size_t fsv_batch_bytes(const fsv_batch *B) { return B ? B->bytes + B->init_bytes : 0; }

size_t fsv_batch_arena_bytes(const fsv_batch *B) { return B ? B->arena_bytes : 0; }

}  // extern "C"

namespace {
// The caller's arena for this call: a different block than the captured
// graph's drops that graph.
// Make instance `instance`'s initial-state list (idx, val) current: the
// concatenated lists of all instances are uploaded into new device buffers
// first, and only when that succeeded do the old buffers go, the instances
// point at their parts and the captured graph (which names the old lists) is
// dropped.  On failure nothing changes.
int replace_init_list(fsv_batch &B, int instance, std::vector<int64_t> &&idx, std::vector<double> &&val) {
    std::vector<BInst> inst = B.inst;
    int64_t total = 0;
    for (int i = 0; i < B.count; ++i) {
        const size_t n = i == instance ? idx.size() : B.init_idx[i].size();
        inst[i].off_init = total;
        inst[i].n_init = (int32_t)n;
        total += (int64_t)n;
    }
    int64_t *d_idx = nullptr;
    double *d_val = nullptr;
    if (total > 0) {
        std::vector<int64_t> hidx;
        std::vector<double> hval;
        hidx.reserve(total);
        hval.reserve(total);
        for (int i = 0; i < B.count; ++i) {
            const std::vector<int64_t> &si = i == instance ? idx : B.init_idx[i];
            const std::vector<double> &sv = i == instance ? val : B.init_val[i];
            hidx.insert(hidx.end(), si.begin(), si.end());
            hval.insert(hval.end(), sv.begin(), sv.end());
        }
        if (hipMalloc((void **)&d_idx, 8 * (size_t)total) != hipSuccess ||
            hipMalloc((void **)&d_val, 8 * (size_t)total) != hipSuccess) {
            (void)hipGetLastError();
            if (d_idx) (void)hipFree(d_idx);
            return fail(FSV_ENOMEM, "hipMalloc of the initial-state lists failed");
        }
        if (hipMemcpy(d_idx, hidx.data(), 8 * (size_t)total, hipMemcpyHostToDevice) != hipSuccess ||
            hipMemcpy(d_val, hval.data(), 8 * (size_t)total, hipMemcpyHostToDevice) != hipSuccess) {
            const hipError_t e = hipGetLastError();
            (void)hipFree(d_idx);
            (void)hipFree(d_val);
            return fail(FSV_EDEVICE, "upload of the initial-state lists failed: %s", hipGetErrorString(e));
        }
    }
    // the new lists are on the device: retire the old ones and switch over
    if (B.work) BHIP(hipStreamSynchronize(B.work));
    if (B.graph) (void)hipGraphExecDestroy(B.graph);
    B.graph = nullptr;
    if (B.d_init_idx) (void)hipFree(B.d_init_idx);
    if (B.d_init_val) (void)hipFree(B.d_init_val);
    B.d_init_idx = d_idx;
    B.d_init_val = d_val;
    B.init_bytes = 16 * (size_t)total;
    B.n_init_total = total;
    B.init_idx[instance] = std::move(idx);
    B.init_val[instance] = std::move(val);
    B.inst = std::move(inst);
    BHIP(hipMemcpy(B.d_inst, B.inst.data(), sizeof(BInst) * B.inst.size(), hipMemcpyHostToDevice));
    return FSV_OK;
}

int bind_arena(fsv_batch &B, void *arena) {
    if (!arena) return fail(FSV_EINVAL, "arena_dev is NULL");
    if ((uintptr_t)arena & 255) return fail(FSV_EINVAL, "the arena must be 256-byte aligned");
    if ((double *)arena != B.d_arena) {
        if (B.work) BHIP(hipStreamSynchronize(B.work));
        if (B.graph) (void)hipGraphExecDestroy(B.graph);
        B.graph = nullptr;
        B.d_arena = (double *)arena;
    }
    return FSV_OK;
}
}  // namespace

extern "C" {

int fsv_batch_energy_grad(fsv_batch *B, const double *theta, void *arena_dev, double *E_out, double *grad_out) {
    if (!B) return fail(FSV_EINVAL, "batch is NULL");
    if (B->total_k > 0 && (!theta || !grad_out)) return fail(FSV_EINVAL, "theta and grad_out are required");
    if (!E_out) return fail(FSV_EINVAL, "E_out is NULL");
    int rc = bind_arena(*B, arena_dev);
    if (rc) return rc;
    return run(*B, theta, E_out, grad_out);
}

int fsv_batch_set_initial_state(fsv_batch *B, int32_t instance, int32_t n_det, const uint64_t *dets,
                                const double *coef) {
    if (!B) return fail(FSV_EINVAL, "batch is NULL");
    if (instance < 0 || instance >= B->count) return fail(FSV_EINVAL, "instance %d of %d", instance, B->count);
    if (n_det < 0 || (n_det > 0 && (!dets || !coef))) return fail(FSV_EINVAL, "bad n_det / dets / coef");
    const BInst &I = B->inst[instance];
    if ((int64_t)n_det > I.dim) return fail(FSV_EINVAL, "more determinants than the sector holds");
    for (int d = 0; d < n_det; ++d)
        if (!std::isfinite(coef[d])) return fail(FSV_ENONFINITE, "non-finite coefficient %d", d);
    const int nq = B->shape[instance][0], na = B->shape[instance][1], nb = B->shape[instance][2];
    const int ordering = B->shape[instance][3], M = nq / 2;
    auto qubit = [&](int so) { return ordering == 0 ? so : so / 2 + (so % 2) * M; };
    const std::vector<uint32_t> sa = strings_of(M, na), sb = strings_of(M, nb);
    std::vector<int32_t> ra((size_t)1 << M, -1), rb((size_t)1 << M, -1);
    for (size_t t = 0; t < sa.size(); ++t) ra[sa[t]] = (int32_t)t;
    for (size_t t = 0; t < sb.size(); ++t) rb[sb[t]] = (int32_t)t;
    std::vector<int64_t> idx(n_det);
    std::vector<double> val(n_det);
    for (int d = 0; d < n_det; ++d) {
        const uint64_t x = dets[d];
        if ((x >> nq) != 0) return fail(FSV_EINVAL, "determinant %d has bits above qubit %d", d, nq - 1);
        uint32_t a = 0, b = 0;
        for (int p = 0; p < M; ++p) {
            a |= (uint32_t)((x >> qubit(2 * p)) & 1u) << p;
            b |= (uint32_t)((x >> qubit(2 * p + 1)) & 1u) << p;
        }
        if (ra[a] < 0 || rb[b] < 0)
            return fail(FSV_EINVAL, "determinant %d lies outside the (%d, %d) sector", d, na, nb);
        idx[d] = (int64_t)ra[a] * I.nsb + rb[b];
        // alpha-first sector amplitude = qubit-basis amplitude x the
        // determinant's reordering sign
        val[d] = (__builtin_popcount(a & beta_prefix_parity(M, ordering, b)) & 1) ? -coef[d] : coef[d];
    }
    {
        std::vector<int64_t> srt(idx);
        std::sort(srt.begin(), srt.end());
        for (size_t t = 1; t < srt.size(); ++t)
            if (srt[t] == srt[t - 1]) return fail(FSV_EINVAL, "a determinant is listed twice");
    }
    const int rc = replace_init_list(*B, instance, std::move(idx), std::move(val));
    if (rc) return rc;
    clear_error();
    return FSV_OK;
}

int fsv_batch_autotune(fsv_batch *B, void *arena_dev, const char **report) {
    static thread_local std::string rep;
    if (!B) return fail(FSV_EINVAL, "batch is NULL");
    if (int rc = bind_arena(*B, arena_dev)) return rc;
    std::vector<double> th(B->total_k, 0.1), e(B->count), g(B->total_k);
    {
        int rc = run(*B, th.data(), e.data(), g.data());  // also leaves valid angles on the device
        if (rc) return rc;
    }
    // candidates: persistent kernel (workgroup size x workgroups per CU) and
    // phased launches (workgroups per instance per rotation launch); both with
    // the LDS budget of a sigma workgroup, which sets the chunk of alpha
    // excitations staged per pass
    struct Cand { int mode, block, per_cu, gx; size_t lds; };
    std::vector<Cand> cands;
    for (size_t lds : {32768, 65536, 98304, 147456}) {
        if (lds > B->lds_max) continue;
        for (int blk : {256, 512, 1024})
            for (int per : {1, 2}) cands.push_back({0, blk, per, B->gx, lds});
        for (int gx : {8, 16, 32, 64})
            if ((size_t)gx <= B->part_cap) cands.push_back({1, B->block, B->per_cu, gx, lds});
        if (B->pk_ok) cands.push_back({2, B->block, B->per_cu, B->gx, lds});
    }
    float best = 1e30f;
    const Cand keep{B->mode, B->block, B->per_cu, B->gx, B->lds_budget};
    Cand bestc = keep;
    hipEvent_t e0, e1;
    BHIP(hipEventCreate(&e0));
    BHIP(hipEventCreate(&e1));
    rep.clear();
    char line[160];
    auto apply = [&](const Cand &c) {
        B->mode = c.mode;
        B->block = c.block;
        B->per_cu = c.per_cu;
        B->gx = c.gx;
        if (B->graph) (void)hipGraphExecDestroy(B->graph);
        B->graph = nullptr;
        return set_lds_budget(*B, c.lds);
    };
    int rc = FSV_OK;
    for (const Cand &c : cands) {
        if ((rc = apply(c))) break;
        float ms = 1e30f;
        for (int r = 0; r < 3 && !rc; ++r) {  // the first run also captures the graph
            float t = 0.f;
            if (hipEventRecord(e0, B->work) != hipSuccess) rc = fail(FSV_EDEVICE, "event record failed");
            if (!rc) rc = launch(*B);
            if (!rc && (hipEventRecord(e1, B->work) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&t, e0, e1) != hipSuccess))
                rc = fail(FSV_EDEVICE, "event timing failed");
            if (r > 0) ms = std::min(ms, t);
        }
        if (rc) break;
        if (c.mode == 0)
            snprintf(line, sizeof line, "persistent: block %d x %d per CU, LDS %zu KiB: %.3f ms\n", c.block,
                     c.per_cu, c.lds / 1024, ms);
        else if (c.mode == 2)
            snprintf(line, sizeof line, "packet runs (%d launches per sweep), LDS %zu KiB: %.3f ms\n", B->pk.runs,
                     c.lds / 1024, ms);
        else
            snprintf(line, sizeof line, "phased: %d workgroups per instance, LDS %zu KiB: %.3f ms\n", c.gx,
                     c.lds / 1024, ms);
        rep += line;
        if (ms < best) {
            best = ms;
            bestc = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    const int rc2 = apply(rc ? keep : bestc);
    if (rc) return rc;
    if (rc2) return rc2;
    snprintf(line, sizeof line, "chosen: %s block %d per_cu %d gx %d LDS %zu KiB\n",
             bestc.mode == 2 ? "packet runs" : (bestc.mode ? "phased" : "persistent"), bestc.block, bestc.per_cu,
             bestc.gx, bestc.lds / 1024);
    rep += line;
    if (report) *report = rep.c_str();
    return FSV_OK;
}

}  // extern "C"
