// Batched evaluation: many independent instances (own qubit count, electrons,
// integrals and operators), each getting energy + adjoint gradient, in one
// persistent kernel launched from a captured HIP graph.
//
// Each instance is processed by one workgroup on its (N_alpha, N_beta) sector
// only, stored compactly as C[Ia][Ib] in the alpha-string-first product basis
// (the JW basis of the blocked qubit ordering restricted to the sector).  In
// that basis an excitation factorises into an alpha part and a beta part:
// tau|Ia Ib> = sign0 * s_a * s_b |Ia' Ib'>, so its active pairs are the
// product of an alpha pair list and a beta pair list (or "all strings" when
// the operator has no alpha / beta part).  Workgroups take instances from a
// device counter in order of decreasing cost.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "../../include/fsv.h"
#include "fsv_internal.h"

using namespace fsv;

namespace {

struct BInst {
    int32_t M, nsa, nsb, nexcA, nexcB, K, ref, pad;
    int64_t dim;
    int64_t off_state;  // double2 offset of psi in the arena; lam follows psi
    int64_t off_ops;    // first BOp
    int64_t off_k;      // first angle / gradient slot
    int64_t off_g;      // first double of (pq|rs)
    int64_t off_ha, off_hb;    // first row pointer of the alpha / beta string Hamiltonian
    int64_t off_excA, off_excB;
    double ecore;
};

using BOp = PairOp;

constexpr int kWave = 64;

__device__ double bsum(double v, double *red) {
    const int lane = threadIdx.x % kWave, wid = threadIdx.x / kWave;
    const int nw = (blockDim.x + kWave - 1) / kWave;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    if (lane == 0) red[wid] = v;
    __syncthreads();
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += red[w];
    __syncthreads();
    return s;
}

__device__ inline void pair_of(const BInst &I, const BOp &op, const uint32_t *__restrict__ lists,
                               int64_t t, int64_t nb, int64_t &src, int64_t &dst, bool &neg) {
    const int64_t u = t / nb, v = t - u * nb;
    int64_t ia = u, ia2 = u, ib = v, ib2 = v;
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
    src = ia * I.nsb + ib;
    dst = ia2 * I.nsb + ib2;
    neg = n;
}

__global__ __launch_bounds__(1024) void k_batch(
    const BInst *__restrict__ inst, const int *__restrict__ order, int count, int *counter,
    const BOp *__restrict__ ops, const uint32_t *__restrict__ lists, const double *__restrict__ cs,
    const double *__restrict__ gint, const int64_t *__restrict__ hptr,
    const int32_t *__restrict__ hcol, const double *__restrict__ hval,
    const uint32_t *__restrict__ exc, double2 *__restrict__ arena, double *__restrict__ grad,
    double *__restrict__ eout) {
    __shared__ int s_idx;
    __shared__ double red[1024 / kWave];
    for (;;) {
        if (threadIdx.x == 0) s_idx = atomicAdd(counter, 1);
        __syncthreads();
        const int idx = s_idx;
        __syncthreads();
        if (idx >= count) break;  // every wave of the workgroup leaves here
        const BInst I = inst[order[idx]];
        double2 *psi = arena + I.off_state;
        double2 *lam = psi + I.dim;
        const int64_t dim = I.dim;

        for (int64_t t = threadIdx.x; t < dim; t += blockDim.x) psi[t] = make_double2(0.0, 0.0);
        __syncthreads();
        if (threadIdx.x == 0) psi[I.ref] = make_double2(1.0, 0.0);
        __syncthreads();

        // forward sweep
        for (int k = 0; k < I.K; ++k) {
            const BOp op = ops[I.off_ops + k];
            const double c = cs[2 * (I.off_k + k)], s = cs[2 * (I.off_k + k) + 1];
            const int64_t na = op.nA >= 0 ? op.nA : I.nsa, nb = op.nB >= 0 ? op.nB : I.nsb;
            for (int64_t t = threadIdx.x; t < na * nb; t += blockDim.x) {
                int64_t xs, xd;
                bool neg;
                pair_of(I, op, lists, t, nb, xs, xd, neg);
                const double sg = neg ? -s : s;
                const double2 a = psi[xs], b = psi[xd];
                psi[xs] = make_double2(c * a.x - sg * b.x, c * a.y - sg * b.y);
                psi[xd] = make_double2(c * b.x + sg * a.x, c * b.y + sg * a.y);
            }
            __syncthreads();
        }

        // lam = H psi on the sector, and E = Re<psi|lam>
        const int M2 = I.M * I.M;
        const double *g = gint + I.off_g;
        const int64_t *pa = hptr + I.off_ha, *pb = hptr + I.off_hb;
        const uint32_t *ea = exc + I.off_excA, *eb = exc + I.off_excB;
        double eacc = 0.0;
        for (int64_t t = threadIdx.x; t < dim; t += blockDim.x) {
            const int64_t Ia = t / I.nsb, Ib = t - Ia * I.nsb;
            const double2 x0 = psi[t];
            double ar = I.ecore * x0.x, ai = I.ecore * x0.y;
            for (int64_t q = pa[Ia]; q < pa[Ia + 1]; ++q) {
                const double v = hval[q];
                const double2 x = psi[(int64_t)hcol[q] * I.nsb + Ib];
                ar += v * x.x;
                ai += v * x.y;
            }
            for (int64_t q = pb[Ib]; q < pb[Ib + 1]; ++q) {
                const double v = hval[q];
                const double2 x = psi[Ia * I.nsb + hcol[q]];
                ar += v * x.x;
                ai += v * x.y;
            }
            for (int e = 0; e < I.nexcA; ++e) {
                const uint32_t wa = ea[Ia * I.nexcA + e];
                const int64_t Ja = wa & 0xFFFFu;
                const double *gp = g + ((wa >> 16) & 0x1FFu) * M2;
                double br = 0.0, bi = 0.0;
                for (int f = 0; f < I.nexcB; ++f) {
                    const uint32_t wb = eb[Ib * I.nexcB + f];
                    const double gv = (wb >> 31) ? -gp[(wb >> 16) & 0x1FFu] : gp[(wb >> 16) & 0x1FFu];
                    const double2 x = psi[Ja * I.nsb + (wb & 0xFFFFu)];
                    br += gv * x.x;
                    bi += gv * x.y;
                }
                if (wa >> 31) {
                    ar -= br;
                    ai -= bi;
                } else {
                    ar += br;
                    ai += bi;
                }
            }
            lam[t] = make_double2(ar, ai);
            eacc += x0.x * ar + x0.y * ai;
        }
        const double E = bsum(eacc, red);

        // reverse adjoint sweep
        for (int k = I.K - 1; k >= 0; --k) {
            const BOp op = ops[I.off_ops + k];
            const double c = cs[2 * (I.off_k + k)], s = cs[2 * (I.off_k + k) + 1];
            const int64_t na = op.nA >= 0 ? op.nA : I.nsa, nb = op.nB >= 0 ? op.nB : I.nsb;
            double acc = 0.0;
            for (int64_t t = threadIdx.x; t < na * nb; t += blockDim.x) {
                int64_t xs, xd;
                bool neg;
                pair_of(I, op, lists, t, nb, xs, xd, neg);
                const double2 a = psi[xs], b = psi[xd], la = lam[xs], lb = lam[xd];
                const double o = lb.x * a.x + lb.y * a.y - la.x * b.x - la.y * b.y;
                acc += neg ? -o : o;
                const double sg = neg ? -s : s;
                psi[xs] = make_double2(c * a.x + sg * b.x, c * a.y + sg * b.y);
                psi[xd] = make_double2(c * b.x - sg * a.x, c * b.y - sg * a.y);
                lam[xs] = make_double2(c * la.x + sg * lb.x, c * la.y + sg * lb.y);
                lam[xd] = make_double2(c * lb.x - sg * la.x, c * lb.y - sg * la.y);
            }
            const double gk = bsum(acc, red);  // also orders this op before the next
            if (threadIdx.x == 0) grad[I.off_k + k] = 2.0 * gk;
        }
        if (threadIdx.x == 0) eout[order[idx]] = E;
        __syncthreads();
    }
}

// ------------------------------------------------------- phased mode ----
// One launch per phase and operator index across all instances: workgroup
// (x, y) serves instance y, x of gridDim.x slices.  Kernel boundaries order
// the phases; no workgroup ever waits on another.

__device__ inline double2 sigma_elem(const BInst &I, const double2 *__restrict__ psi, int64_t t,
                                     const double *__restrict__ gint, const int64_t *__restrict__ hptr,
                                     const int32_t *__restrict__ hcol, const double *__restrict__ hval,
                                     const uint32_t *__restrict__ exc) {
    const int M2 = I.M * I.M;
    const double *g = gint + I.off_g;
    const int64_t *pa = hptr + I.off_ha, *pb = hptr + I.off_hb;
    const uint32_t *ea = exc + I.off_excA, *eb = exc + I.off_excB;
    const int64_t Ia = t / I.nsb, Ib = t - Ia * I.nsb;
    const double2 x0 = psi[t];
    double ar = I.ecore * x0.x, ai = I.ecore * x0.y;
    for (int64_t q = pa[Ia]; q < pa[Ia + 1]; ++q) {
        const double v = hval[q];
        const double2 x = psi[(int64_t)hcol[q] * I.nsb + Ib];
        ar += v * x.x;
        ai += v * x.y;
    }
    for (int64_t q = pb[Ib]; q < pb[Ib + 1]; ++q) {
        const double v = hval[q];
        const double2 x = psi[Ia * I.nsb + hcol[q]];
        ar += v * x.x;
        ai += v * x.y;
    }
    for (int e = 0; e < I.nexcA; ++e) {
        const uint32_t wa = ea[Ia * I.nexcA + e];
        const int64_t Ja = wa & 0xFFFFu;
        const double *gp = g + ((wa >> 16) & 0x1FFu) * M2;
        double br = 0.0, bi = 0.0;
        for (int f = 0; f < I.nexcB; ++f) {
            const uint32_t wb = eb[Ib * I.nexcB + f];
            const double gv = (wb >> 31) ? -gp[(wb >> 16) & 0x1FFu] : gp[(wb >> 16) & 0x1FFu];
            const double2 x = psi[Ja * I.nsb + (wb & 0xFFFFu)];
            br += gv * x.x;
            bi += gv * x.y;
        }
        if (wa >> 31) {
            ar -= br;
            ai -= bi;
        } else {
            ar += br;
            ai += bi;
        }
    }
    return make_double2(ar, ai);
}

__global__ __launch_bounds__(256) void k_pinit(const BInst *__restrict__ inst, double2 *__restrict__ arena) {
    const BInst I = inst[blockIdx.y];
    double2 *psi = arena + I.off_state;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < I.dim;
         t += (int64_t)gridDim.x * blockDim.x)
        psi[t] = make_double2(t == I.ref ? 1.0 : 0.0, 0.0);
}

__global__ __launch_bounds__(256) void k_pfwd(const BInst *__restrict__ inst, const BOp *__restrict__ ops,
                                              const uint32_t *__restrict__ lists,
                                              const double *__restrict__ cs, double2 *__restrict__ arena,
                                              int k) {
    const BInst I = inst[blockIdx.y];
    if (k >= I.K) return;
    const BOp op = ops[I.off_ops + k];
    const double c = cs[2 * (I.off_k + k)], s = cs[2 * (I.off_k + k) + 1];
    double2 *psi = arena + I.off_state;
    const int64_t na = op.nA >= 0 ? op.nA : I.nsa, nb = op.nB >= 0 ? op.nB : I.nsb;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < na * nb;
         t += (int64_t)gridDim.x * blockDim.x) {
        int64_t xs, xd;
        bool neg;
        pair_of(I, op, lists, t, nb, xs, xd, neg);
        const double sg = neg ? -s : s;
        const double2 a = psi[xs], b = psi[xd];
        psi[xs] = make_double2(c * a.x - sg * b.x, c * a.y - sg * b.y);
        psi[xd] = make_double2(c * b.x + sg * a.x, c * b.y + sg * a.y);
    }
}

__global__ __launch_bounds__(256) void k_psigma(const BInst *__restrict__ inst, const double *__restrict__ gint,
                                                const int64_t *__restrict__ hptr,
                                                const int32_t *__restrict__ hcol,
                                                const double *__restrict__ hval,
                                                const uint32_t *__restrict__ exc,
                                                double2 *__restrict__ arena, double *__restrict__ epart) {
    __shared__ double red[256 / kWave];
    const BInst I = inst[blockIdx.y];
    const double2 *psi = arena + I.off_state;
    double2 *lam = arena + I.off_state + I.dim;
    double acc = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < I.dim;
         t += (int64_t)gridDim.x * blockDim.x) {
        const double2 v = sigma_elem(I, psi, t, gint, hptr, hcol, hval, exc);
        lam[t] = v;
        const double2 x0 = psi[t];
        acc += x0.x * v.x + x0.y * v.y;
    }
    acc = bsum(acc, red);
    if (threadIdx.x == 0) epart[(int64_t)blockIdx.y * gridDim.x + blockIdx.x] = acc;
}

__global__ __launch_bounds__(256) void k_prev(const BInst *__restrict__ inst, const BOp *__restrict__ ops,
                                              const uint32_t *__restrict__ lists,
                                              const double *__restrict__ cs, double2 *__restrict__ arena,
                                              int k, double *__restrict__ gpart) {
    __shared__ double red[256 / kWave];
    const BInst I = inst[blockIdx.y];
    if (k >= I.K) return;  // uniform across the workgroup
    const BOp op = ops[I.off_ops + k];
    const double c = cs[2 * (I.off_k + k)], s = cs[2 * (I.off_k + k) + 1];
    double2 *psi = arena + I.off_state;
    double2 *lam = psi + I.dim;
    const int64_t na = op.nA >= 0 ? op.nA : I.nsa, nb = op.nB >= 0 ? op.nB : I.nsb;
    double acc = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < na * nb;
         t += (int64_t)gridDim.x * blockDim.x) {
        int64_t xs, xd;
        bool neg;
        pair_of(I, op, lists, t, nb, xs, xd, neg);
        const double2 a = psi[xs], b = psi[xd], la = lam[xs], lb = lam[xd];
        const double o = lb.x * a.x + lb.y * a.y - la.x * b.x - la.y * b.y;
        acc += neg ? -o : o;
        const double sg = neg ? -s : s;
        psi[xs] = make_double2(c * a.x + sg * b.x, c * a.y + sg * b.y);
        psi[xd] = make_double2(c * b.x - sg * a.x, c * b.y - sg * a.y);
        lam[xs] = make_double2(c * la.x + sg * lb.x, c * la.y + sg * lb.y);
        lam[xd] = make_double2(c * lb.x - sg * la.x, c * lb.y - sg * la.y);
    }
    acc = bsum(acc, red);
    if (threadIdx.x == 0) gpart[(I.off_k + k) * gridDim.x + blockIdx.x] = acc;
}

// Ordered per-instance sums of the partials: E and 2 * per-operator sums.
__global__ __launch_bounds__(64) void k_preduce(const BInst *__restrict__ inst, int gx,
                                                const double *__restrict__ epart,
                                                const double *__restrict__ gpart,
                                                double *__restrict__ grad, double *__restrict__ eout) {
    const int y = blockIdx.x;
    const BInst I = inst[y];
    if (threadIdx.x == 0) {
        double e = 0.0;
        for (int x = 0; x < gx; ++x) e += epart[(int64_t)y * gx + x];
        eout[y] = e;
    }
    for (int k = threadIdx.x; k < I.K; k += blockDim.x) {
        double s = 0.0;
        for (int x = 0; x < gx; ++x) s += gpart[(I.off_k + k) * gx + x];
        grad[I.off_k + k] = 2.0 * s;
    }
}

__global__ void k_zero_int(int *p) {
    if (threadIdx.x == 0 && blockIdx.x == 0) *p = 0;
}

template <typename T>
int dmalloc(std::vector<void *> &owned, T **out, size_t count) {
    void *p = nullptr;
    const size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(FSV_ENOMEM, "hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    }
    owned.push_back(p);
    *out = (T *)p;
    return FSV_OK;
}

}  // namespace

struct fsv_batch {
    int count = 0;
    int64_t total_k = 0;
    std::vector<BInst> inst;
    std::vector<int> order;
    std::vector<void *> owned;
    size_t bytes = 0;
    hipStream_t user = nullptr, work = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    BInst *d_inst = nullptr;
    int *d_order = nullptr, *d_counter = nullptr;
    BOp *d_ops = nullptr;
    uint32_t *d_lists = nullptr, *d_exc = nullptr;
    double *d_cs = nullptr, *d_g = nullptr, *d_hval = nullptr, *d_grad = nullptr, *d_e = nullptr;
    int64_t *d_hptr = nullptr;
    int32_t *d_hcol = nullptr;
    double2 *d_arena = nullptr;
    double *h_pin = nullptr;  // cs (2 total_k) | grad (total_k) | E (count)
    int block = 256, per_cu = 2, cus = 256;
    int mode = 1;       // 0 persistent work-queue kernel, 1 phased launches
    int gx = 32;        // phased mode: workgroups per instance per launch
    int kmax = 0;
    double *d_epart = nullptr, *d_gpart = nullptr;
    size_t part_cap = 0;  // workgroups per instance the partial buffers hold
    bool use_graph = true;
    hipGraphExec_t graph = nullptr;
    ~fsv_batch() {
        if (work) (void)hipStreamSynchronize(work);
        if (graph) (void)hipGraphExecDestroy(graph);
        for (void *p : owned) (void)hipFree(p);
        if (h_pin) (void)hipHostFree(h_pin);
        if (ev_in) (void)hipEventDestroy(ev_in);
        if (ev_out) (void)hipEventDestroy(ev_out);
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

int enqueue(fsv_batch &B) {
    if (B.mode == 1) {
        const dim3 grid((unsigned)B.gx, (unsigned)B.count);
        hipLaunchKernelGGL(k_pinit, grid, dim3(256), 0, B.work, B.d_inst, B.d_arena);
        BHIP(hipGetLastError());
        for (int k = 0; k < B.kmax; ++k) {
            hipLaunchKernelGGL(k_pfwd, grid, dim3(256), 0, B.work, B.d_inst, B.d_ops, B.d_lists, B.d_cs,
                               B.d_arena, k);
            BHIP(hipGetLastError());
        }
        hipLaunchKernelGGL(k_psigma, grid, dim3(256), 0, B.work, B.d_inst, B.d_g, B.d_hptr, B.d_hcol,
                           B.d_hval, B.d_exc, B.d_arena, B.d_epart);
        BHIP(hipGetLastError());
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
    hipLaunchKernelGGL(k_batch, dim3(grid), dim3(B.block), 0, B.work, B.d_inst, B.d_order, B.count,
                       B.d_counter, B.d_ops, B.d_lists, B.d_cs, B.d_g, B.d_hptr, B.d_hcol, B.d_hval,
                       B.d_exc, B.d_arena, B.d_grad, B.d_e);
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
    double *cs = B.h_pin;
    for (int64_t k = 0; k < B.total_k; ++k) {
        if (!std::isfinite(theta[k])) return fail(FSV_ENONFINITE, "non-finite theta at %lld", (long long)k);
        cs[2 * k] = std::cos(theta[k]);
        cs[2 * k + 1] = std::sin(theta[k]);
    }
    BHIP(hipEventRecord(B.ev_in, B.user));
    BHIP(hipStreamWaitEvent(B.work, B.ev_in, 0));
    if (B.total_k)
        BHIP(hipMemcpyAsync(B.d_cs, cs, sizeof(double) * 2 * B.total_k, hipMemcpyHostToDevice, B.work));
    int rc = launch(B);
    if (rc) return rc;
    double *hg = B.h_pin + 2 * B.total_k, *he = hg + B.total_k;
    if (B.total_k)
        BHIP(hipMemcpyAsync(hg, B.d_grad, sizeof(double) * B.total_k, hipMemcpyDeviceToHost, B.work));
    BHIP(hipMemcpyAsync(he, B.d_e, sizeof(double) * B.count, hipMemcpyDeviceToHost, B.work));
    BHIP(hipStreamSynchronize(B.work));
    BHIP(hipEventRecord(B.ev_out, B.work));
    BHIP(hipStreamWaitEvent(B.user, B.ev_out, 0));
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
        if (problems[i].precision != 0) return fail(FSV_EINVAL, "instance %d: batches are complex128 only", i);
        if (problems[i].n_qubits > 30) return fail(FSV_EINVAL, "instance %d: batches take at most 30 qubits", i);
    }
    fsv_batch *B = new (std::nothrow) fsv_batch();
    if (!B) return fail(FSV_ENOMEM, "batch allocation failed");
    B->count = count;
    B->user = (hipStream_t)hip_stream;
    B->use_graph = std::getenv("FSV_NO_GRAPH") == nullptr;
    if (const char *m = std::getenv("FSV_BATCH_MODE")) B->mode = std::strcmp(m, "persistent") == 0 ? 0 : 1;

    std::vector<BOp> ops;
    std::vector<uint32_t> lists, excs;
    std::vector<double> gall, hval;
    std::vector<int64_t> hptr;
    std::vector<int32_t> hcol;
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
        // string Hamiltonians (row pointers are global indices into hcol / hval)
        for (int s = 0; s < 2; ++s) {
            std::vector<int64_t> ptr;
            std::vector<int32_t> col;
            std::vector<double> val;
            build_string_h(M, s ? sb : sa, s ? rb : ra, p.h, p.g, ptr, col, val);
            const int64_t base = (int64_t)hcol.size();
            (s ? I.off_hb : I.off_ha) = (int64_t)hptr.size();
            for (int64_t v : ptr) hptr.push_back(v + base);
            hcol.insert(hcol.end(), col.begin(), col.end());
            hval.insert(hval.end(), val.begin(), val.end());
        }
        std::vector<uint32_t> ea, eb;
        build_exc(M, sa, ra, ea, I.nexcA);
        build_exc(M, sb, rb, eb, I.nexcB);
        I.off_excA = (int64_t)excs.size();
        excs.insert(excs.end(), ea.begin(), ea.end());
        I.off_excB = (int64_t)excs.size();
        excs.insert(excs.end(), eb.begin(), eb.end());
        // operators in the alpha-first basis = the blocked JW ordering
        double pairs = 0.0;
        for (int k = 0; k < p.n_ops; ++k) {
            const BOp o = build_pair_op(M, p.ops + 4 * k, sa, ra, sb, rb, lists);
            pairs += (double)(o.nA >= 0 ? o.nA : I.nsa) * (double)(o.nB >= 0 ? o.nB : I.nsb);
            ops.push_back(o);
        }
        const double nnz = (double)(hptr[I.off_ha + I.nsa] - hptr[I.off_ha]) / std::max(1, I.nsa) +
                           (double)(hptr[I.off_hb + I.nsb] - hptr[I.off_hb]) / std::max(1, I.nsb);
        cost[i] = (double)I.dim * (nnz + (double)I.nexcA * I.nexcB) + 3.0 * pairs;
        B->inst.push_back(I);
    }
    B->total_k = kk;
    for (int i = 0; i < count; ++i) B->kmax = std::max(B->kmax, problems[i].n_ops);
    B->part_cap = 64;
    B->order.resize(count);
    std::iota(B->order.begin(), B->order.end(), 0);
    std::stable_sort(B->order.begin(), B->order.end(), [&](int a, int b) { return cost[a] > cost[b]; });

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
        hipEventCreateWithFlags(&B->ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&B->ev_out, hipEventDisableTiming) != hipSuccess) {
        delete B;
        return fail(FSV_EDEVICE, "stream/event creation failed");
    }
    if (hipHostMalloc((void **)&B->h_pin, sizeof(double) * (3 * kk + count + 8), hipHostMallocDefault) != hipSuccess) {
        delete B;
        return fail(FSV_ENOMEM, "pinned host buffer");
    }
    auto& o = B->owned;
    if ((rc = dmalloc(o, &B->d_inst, B->inst.size())) || (rc = dmalloc(o, &B->d_order, count)) ||
        (rc = dmalloc(o, &B->d_counter, 4)) || (rc = dmalloc(o, &B->d_ops, ops.size())) ||
        (rc = dmalloc(o, &B->d_lists, lists.size())) || (rc = dmalloc(o, &B->d_exc, excs.size())) ||
        (rc = dmalloc(o, &B->d_cs, 2 * (size_t)kk)) || (rc = dmalloc(o, &B->d_g, gall.size())) ||
        (rc = dmalloc(o, &B->d_hval, hval.size())) || (rc = dmalloc(o, &B->d_hptr, hptr.size())) ||
        (rc = dmalloc(o, &B->d_hcol, hcol.size())) || (rc = dmalloc(o, &B->d_grad, (size_t)kk)) ||
        (rc = dmalloc(o, &B->d_e, (size_t)count)) || (rc = dmalloc(o, &B->d_arena, (size_t)state)) ||
        (rc = dmalloc(o, &B->d_epart, (size_t)count * B->part_cap)) ||
        (rc = dmalloc(o, &B->d_gpart, (size_t)kk * B->part_cap)))
        return fin(rc);
    B->bytes = sizeof(BInst) * B->inst.size() + sizeof(int) * (count + 4) + sizeof(BOp) * ops.size() +
               4 * (lists.size() + excs.size()) + 8 * (2 * kk + gall.size() + hval.size() + hptr.size() + kk + count) +
               4 * hcol.size() + 16 * (size_t)state;
    struct Up { void *d; const void *h; size_t n; };
    const Up ups[] = {
        {B->d_inst, B->inst.data(), sizeof(BInst) * B->inst.size()},
        {B->d_order, B->order.data(), sizeof(int) * count},
        {B->d_ops, ops.data(), sizeof(BOp) * ops.size()},
        {B->d_lists, lists.data(), 4 * lists.size()},
        {B->d_exc, excs.data(), 4 * excs.size()},
        {B->d_g, gall.data(), 8 * gall.size()},
        {B->d_hval, hval.data(), 8 * hval.size()},
        {B->d_hptr, hptr.data(), 8 * hptr.size()},
        {B->d_hcol, hcol.data(), 4 * hcol.size()},
    };
    for (const Up &u : ups)
        if (u.n && hipMemcpy(u.d, u.h, u.n, hipMemcpyHostToDevice) != hipSuccess)
            return fin(fail(FSV_EDEVICE, "upload failed"));
    *out = B;
    clear_error();
    return FSV_OK;
}

int fsv_batch_destroy(fsv_batch *B) {
    delete B;
    return FSV_OK;
}

size_t fsv_batch_bytes(const fsv_batch *B) { return B ? B->bytes : 0; }

int fsv_batch_energy_grad(fsv_batch *B, const double *theta, double *E_out, double *grad_out) {
    if (!B) return fail(FSV_EINVAL, "batch is NULL");
    if (B->total_k > 0 && (!theta || !grad_out)) return fail(FSV_EINVAL, "theta and grad_out are required");
    if (!E_out) return fail(FSV_EINVAL, "E_out is NULL");
    return run(*B, theta, E_out, grad_out);
}

int fsv_batch_autotune(fsv_batch *B, const char **report) {
    static thread_local std::string rep;
    if (!B) return fail(FSV_EINVAL, "batch is NULL");
    std::vector<double> th(B->total_k, 0.1), e(B->count), g(B->total_k);
    {
        int rc = run(*B, th.data(), e.data(), g.data());  // also leaves valid angles on the device
        if (rc) return rc;
    }
    // candidates: persistent kernel (workgroup size x workgroups per CU) and
    // phased launches (workgroups per instance)
    struct Cand { int mode, block, per_cu, gx; };
    std::vector<Cand> cands;
    for (int blk : {256, 512, 1024})
        for (int per : {1, 2, 4}) cands.push_back({0, blk, per, B->gx});
    for (int gx : {8, 16, 32, 64})
        if ((size_t)gx <= B->part_cap) cands.push_back({1, B->block, B->per_cu, gx});
    float best = 1e30f;
    Cand bestc{B->mode, B->block, B->per_cu, B->gx};
    hipEvent_t e0, e1;
    BHIP(hipEventCreate(&e0));
    BHIP(hipEventCreate(&e1));
    rep.clear();
    char line[128];
    const bool graph = B->use_graph;
    B->use_graph = false;
    for (const Cand &c : cands) {
        B->mode = c.mode;
        B->block = c.block;
        B->per_cu = c.per_cu;
        B->gx = c.gx;
        float ms = 0.f;
        for (int r = 0; r < 2; ++r) {
            BHIP(hipEventRecord(e0, B->work));
            int rc = enqueue(*B);
            if (rc) return rc;
            BHIP(hipEventRecord(e1, B->work));
            BHIP(hipEventSynchronize(e1));
            BHIP(hipEventElapsedTime(&ms, e0, e1));
        }
        if (c.mode == 0)
            snprintf(line, sizeof line, "persistent: block %d x %d per CU: %.3f ms\n", c.block, c.per_cu, ms);
        else
            snprintf(line, sizeof line, "phased: %d workgroups per instance: %.3f ms\n", c.gx, ms);
        rep += line;
        if (ms < best) {
            best = ms;
            bestc = c;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    B->use_graph = graph;
    B->mode = bestc.mode;
    B->block = bestc.block;
    B->per_cu = bestc.per_cu;
    B->gx = bestc.gx;
    if (B->graph) (void)hipGraphExecDestroy(B->graph);
    B->graph = nullptr;
    snprintf(line, sizeof line, "chosen: %s block %d per_cu %d gx %d\n", bestc.mode ? "phased" : "persistent",
             bestc.block, bestc.per_cu, bestc.gx);
    rep += line;
    if (report) *report = rep.c_str();
    return FSV_OK;
}

}  // extern "C"
