// Host side of the C-ABI library: validation, operator compilation, sector
// string tables, same-spin string Hamiltonians (Slater-Condon rules), graph
// capture of the energy/gradient pass, finite differences and launch tuning.
#include <hip/hip_runtime.h>
#include <rocblas/rocblas.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/fsv.h"
#include "fsv_internal.h"

using namespace fsv;

// ------------------------------------------------------------------ errors --
namespace fsv {
thread_local std::string g_err;

int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

void clear_error() { g_err.clear(); }
}  // namespace fsv

namespace {

#define HIPCHECK(expr)                                                                      \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess)                                                               \
            return fail(FSV_EDEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));        \
    } while (0)

int popcount64(uint64_t v) { return __builtin_popcountll(v); }

// JW action of a^+_q (dag) or a_q on a bit string; 0 when annihilated.
int jw_step(uint64_t &x, bool dag, int q) {
    const uint64_t b = 1ull << q;
    if (dag == ((x & b) != 0)) return 0;
    const int s = (popcount64(x & (b - 1)) & 1) ? -1 : 1;
    x ^= b;
    return s;
}

bool finite_all(const double *a, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(a[i])) return false;
    return true;
}

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

}  // namespace

// ------------------------------------------------------- no-alloc scratch --
// Scratch of energy_grad_noalloc: one block per GPU, part of the library's
// device image, held until the process ends.  Host code never passes the
// array's name to a kernel or a copy: it is a host-side stand-in there.  The
// device address comes from hipGetSymbolAddress, once per device.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

// The current device's scratch address (looked up on its first use).
int scratch_address(void **out) {
    int dev = 0;
    HIPCHECK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(FSV_EDEVICE, "device %d outside the scratch table", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress((void **)&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr) {
            (void)hipGetLastError();
            return fail(FSV_EDEVICE, "hipGetSymbolAddress of the scratch block failed: %s", hipGetErrorString(e));
        }
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return FSV_OK;
}

}  // namespace

// -------------------------------------------------------------------- plan --
struct fsv_plan {
    int n = 0, M = 0, na = 0, nb = 0, ordering = 0, precision = 0, K = 0;
    double ecore = 0.0;
    std::vector<double> h, g, v;
    std::vector<int32_t> ops;
    std::vector<RotOp> rot;
    std::vector<uint64_t> npairs;
    Shape shape_rot{256, 4}, shape_adj{256, 2};
    bool wide = false;   // 64-bit index math
    int amp_bytes = 16;
    uint64_t ref_index = 0;
    double ref_phase = 1.0;  // ordering sign of the reference in the alpha-first basis

    // forward segmentation: fused LDS runs [k0, k1) (k1 - k0 >= 2) or single ops
    struct Seg { int k0, k1; bool fused; };
    std::vector<Seg> segs;
    int tile_bits = 12;

    // sector tables
    int64_t nsa = 0, nsb = 0, dim = 0;
    int nexcA = 0, nexcB = 0;
    std::vector<uint32_t> sa, sb;
    std::vector<int64_t> ha_ptr, hb_ptr;
    std::vector<int32_t> ha_col, hb_col;
    std::vector<double> ha_val, hb_val;

    // device
    hipStream_t user = nullptr, work = nullptr;
    hipEvent_t ev_in = nullptr, ev_out = nullptr;
    // recorded after each angle upload from h_pin: the next upload waits for
    // it before rewriting the pinned angles (fsv_set_theta returns at once)
    hipEvent_t ev_cs = nullptr;
    bool cs_pending = false;
    std::vector<DevBuf> bufs;
    RotOp *d_rot = nullptr;
    double *d_cs = nullptr, *d_gpart = nullptr, *d_epart = nullptr, *d_out = nullptr;
    int *d_gcount = nullptr, *d_ecount = nullptr;
    uint64_t *d_Xa = nullptr, *d_Xb = nullptr;
    uint32_t *d_sa = nullptr, *d_PPb = nullptr, *d_excA = nullptr, *d_excB = nullptr, *d_excBT = nullptr;
    double *d_g = nullptr;
    int64_t *d_ha_ptr = nullptr, *d_hb_ptr = nullptr;
    int32_t *d_ha_col = nullptr, *d_hb_col = nullptr;
    double *d_ha_val = nullptr, *d_hb_val = nullptr;
    // device-side refresh of those values when the one-body potential changes
    double *d_ha_v2 = nullptr, *d_hb_v2 = nullptr, *d_htilde = nullptr;  // two-body parts, h + v
    int32_t *d_ha_desc = nullptr, *d_hb_desc = nullptr;                   // one-body descriptors
    uint32_t *d_str_a = nullptr, *d_str_b = nullptr;                      // string masks
    int32_t *d_binA_off = nullptr, *d_binA_idx = nullptr, *d_binB_off = nullptr, *d_binB_idx = nullptr;
    // Sector workspace: one block, caller-provided (fsv_plan_set_workspace) or
    // allocated by the plan on first use, holding d_C .. d_epart below.
    // d_C also holds the interleaved (psi, lam) pairs of a packet adjoint sweep.
    double2 *d_C = nullptr, *d_S = nullptr, *d_CT = nullptr, *d_ST = nullptr, *d_O = nullptr;
    double2 *d_gamma = nullptr, *d_YT = nullptr;
    void *ws = nullptr;
    bool ws_owned = false, ws_warm = false;
    size_t ws_bytes = 0;
    size_t ws_off[10] = {};  // byte offsets of C, S, CT, ST, O, gamma, YT, gpart, epart; [9] = end
    // the parts energy_grad_noalloc takes from the scratch block (sector
    // engine): C, S, CT, ST, YT, gpart, epart offsets; [7] = end
    size_t na_off[8] = {};
    double *h_pin = nullptr;  // pinned: cs (2K) then out (K + 1) then gamma (4 M^2)
    double *h_cs = nullptr;   // pinned, coherent: cs (2K) read by energy_grad's graph itself
    size_t pin_doubles = 0;

    // sector-compressed engine (default for energy_grad / ansatz_apply)
    int engine = 0;  // 0 sector-compressed, 1 dense
    int excitation = 0;  // 0 fermionic, 1 qubit excitations
    // multi-determinant start (n_init = 0: the reference determinant):
    // sector index and signed value for the sector engine, qubit index and
    // value for the dense engine
    int n_init = 0;
    int64_t *d_init_sidx = nullptr, *d_init_didx = nullptr;
    double *d_init_sval = nullptr, *d_init_dval = nullptr;
    std::vector<void *> init_mem;
    std::vector<uint32_t> PPb;  // per-beta-string prefix parity (host copy)
    int svt = V_F64;  // storage of the sector state: real FP64, or real FP32 for precision 1
    SectorTabs tabs{};
    int lr_R = 0;     // rank of the factorised alpha-beta product (0: direct)
    // dense same-spin string Hamiltonians (FP64 GEMM on the matrix cores)
    rocblas_handle blas = nullptr;
    double *d_ha_dense = nullptr, *d_hb_dense = nullptr, *d_hb_dense_t = nullptr;
    std::vector<PairOp> pops;
    std::vector<uint32_t> h_plists;  // host copy of the pair lists (fused-run tables are built from it)
    uint32_t *d_plists = nullptr;
    PairOp *d_pops = nullptr;
    int *d_ccount = nullptr;
    // fused operator runs of the forward and adjoint sweeps (LDS budget per tile)
    FusedSched ffwd, frev;
    size_t fuse_budget_fwd = 65536, fuse_budget_rev = 98304;
    // 0 LDS tiles where the cost model gains, 1 never (FSV_NO_FUSE), 2 every tile
    // run (FSV_FORCE_FUSE), 3 component packets (the default for states of at
    // most packet_default_dim() amplitudes, where the cost model decides)
    int fuse_mode = 0;

    // graphs
    uint64_t gen = 0;  // bumped whenever captured launches may have changed
    bool use_graph = true;
    bool defer_e = false;  // energy_grad body: E is reduced with the gradients, after the sweep
    // energy_grad body, real FP64 state, adjoint sweep on pairs: the product
    // may write lam interleaved with psi into d_C (z_ready then says so)
    bool zip_in_sigma = false, z_ready = false;
    hipGraphExec_t g_eg = nullptr;
    const void *g_eg_psi = nullptr, *g_eg_lam = nullptr;
    hipGraphExec_t g_e = nullptr;
    const void *g_e_psi = nullptr;

    // pools compiled for this plan and still alive: a plan destroyed first
    // detaches them (they then refuse to run), so a pool never reads a freed plan
    std::vector<fsv_pool *> pools;

    ~fsv_plan();
};

// An operator pool compiled for one plan's sector (ADAPT screening).  plan is
// nullptr once that plan has been destroyed.
struct fsv_pool {
    fsv_plan *plan = nullptr;
    int n = 0, gx = 1;
    PairOp *d_ops = nullptr;
    uint32_t *d_lists = nullptr;
    double *d_part = nullptr, *d_out = nullptr;
    int *d_counts = nullptr;
    double *h_pin = nullptr;  // E, then the n screening values
    hipGraphExec_t graph = nullptr;
    const void *g_psi = nullptr, *g_lam = nullptr;
    uint64_t gen = 0;
    std::vector<void *> mem;
    ~fsv_pool() {
        if (graph) (void)hipGraphExecDestroy(graph);
        for (void *p : mem) (void)hipFree(p);
        if (h_pin) (void)hipHostFree(h_pin);
    }
};

namespace {

int qubit_of(const fsv_plan &P, int so) {
    const int p = so / 2, s = so % 2;
    return P.ordering == 0 ? so : p + s * P.M;
}

template <typename T>
int dalloc(fsv_plan &P, T **out, size_t count) {
    size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(FSV_ENOMEM, "hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
    }
    P.bufs.push_back({p, bytes});
    *out = (T *)p;
    return FSV_OK;
}

template <typename T>
int upload(fsv_plan &P, T *dst, const T *src, size_t count) {
    if (count == 0) return FSV_OK;
    HIPCHECK(hipMemcpyAsync(dst, src, count * sizeof(T), hipMemcpyHostToDevice, P.work));
    HIPCHECK(hipStreamSynchronize(P.work));
    return FSV_OK;
}

}  // namespace

int fsv::validate_problem(const fsv_problem *p) {
    if (!p) return fail(FSV_EINVAL, "problem is NULL");
    if (p->n_qubits < 2 || p->n_qubits > 34 || (p->n_qubits & 1))
        return fail(FSV_EINVAL, "n_qubits must be even and in 2..34 (got %d)", p->n_qubits);
    const int M = p->n_qubits / 2;
    if (p->n_alpha < 0 || p->n_alpha > M || p->n_beta < 0 || p->n_beta > M)
        return fail(FSV_EINVAL, "n_alpha/n_beta out of range 0..%d", M);
    if (p->ordering != 0 && p->ordering != 1) return fail(FSV_EINVAL, "ordering must be 0 or 1");
    if (p->precision != 0 && p->precision != 1) return fail(FSV_EINVAL, "precision must be 0 or 1");
    if (!p->h || !p->g) return fail(FSV_EINVAL, "h and g are required");
    if (p->n_ops < 0 || (p->n_ops > 0 && !p->ops)) return fail(FSV_EINVAL, "bad n_ops/ops");
    const size_t M2 = (size_t)M * M, M4 = M2 * M2;
    if (!finite_all(p->h, M2) || !finite_all(p->g, M4) || !std::isfinite(p->e_core))
        return fail(FSV_ENONFINITE, "non-finite value in h, g or e_core");
    double scale = 0.0;
    for (size_t i = 0; i < M4; ++i) scale = std::max(scale, std::fabs(p->g[i]));
    for (size_t i = 0; i < M2; ++i) scale = std::max(scale, std::fabs(p->h[i]));
    const double tol = 1e-12 * std::max(1.0, scale);
    for (int a = 0; a < M; ++a)
        for (int b = 0; b < M; ++b)
            if (std::fabs(p->h[a * M + b] - p->h[b * M + a]) > tol)
                return fail(FSV_EINVAL, "h is not symmetric at (%d,%d)", a, b);
    for (int q = 0; q < M; ++q)
        for (int r = 0; r < M; ++r)
            for (int s = 0; s < M; ++s)
                for (int t = 0; t < M; ++t) {
                    const double x = p->g[((q * M + r) * M + s) * M + t];
                    const double y1 = p->g[((r * M + q) * M + s) * M + t];
                    const double y2 = p->g[((q * M + r) * M + t) * M + s];
                    const double y3 = p->g[((s * M + t) * M + q) * M + r];
                    if (std::fabs(x - y1) > tol || std::fabs(x - y2) > tol || std::fabs(x - y3) > tol)
                        return fail(FSV_EINVAL, "g lacks 8-fold symmetry at (%d%d|%d%d)", q, r, s, t);
                }
    if (p->excitation != 0 && p->excitation != 1) return fail(FSV_EINVAL, "excitation must be 0 or 1");
    return validate_ops(p->n_qubits, p->n_ops, p->ops);
}

int fsv::validate_ops(int n, int n_ops, const int32_t *ops) {
    if (n_ops < 0 || (n_ops > 0 && !ops)) return fail(FSV_EINVAL, "bad n_ops/ops");
    for (int k = 0; k < n_ops; ++k) {
        const int32_t *o = ops + 4 * k;
        const int a = o[0], b = o[1], j = o[2], i = o[3];
        const bool single = (b < 0);
        if (single) {
            if (j >= 0 || b != -1 || j != -1)
                return fail(FSV_EINVAL, "op %d: a single excitation has b = j = -1", k);
            if (a < 0 || a >= n || i < 0 || i >= n || a == i)
                return fail(FSV_EINVAL, "op %d: indices out of range or repeated", k);
            if ((a & 1) != (i & 1)) return fail(FSV_EINVAL, "op %d: spin-flip excitation", k);
        } else {
            if (a < 0 || a >= n || b < 0 || b >= n || j < 0 || j >= n || i < 0 || i >= n)
                return fail(FSV_EINVAL, "op %d: index out of range", k);
            if (a == b || a == j || a == i || b == j || b == i || j == i)
                return fail(FSV_EINVAL, "op %d: repeated index", k);
            const int up_c = ((a & 1) == 0) + ((b & 1) == 0);
            const int up_a = ((i & 1) == 0) + ((j & 1) == 0);
            if (up_c != up_a) return fail(FSV_EINVAL, "op %d: does not conserve alpha/beta counts", k);
        }
    }
    return FSV_OK;
}

// Compile one operator for a given qubit ordering: sorted target qubits,
// source/destination patterns, the parity mask of non-target bits and the
// constant sign of the JW string of tau (excitation 1: a qubit excitation,
// sign +1 on every pair).
RotOp fsv::compile_op(int M, int ordering, const int32_t *o, int excitation) {
    auto qubit = [&](int so) { return ordering == 0 ? so : so / 2 + (so % 2) * M; };
    RotOp r{};
    const bool single = o[1] < 0;
    const int qa = qubit(o[0]), qi = qubit(o[3]);
    int qs[4], nt = 0;
    uint64_t src = 1ull << qi, dst = 1ull << qa;
    uint64_t par = ((1ull << qi) - 1) ^ ((1ull << qa) - 1);
    qs[nt++] = qi;
    qs[nt++] = qa;
    int qb = -1, qj = -1;
    if (!single) {
        qb = qubit(o[1]);
        qj = qubit(o[2]);
        src |= 1ull << qj;
        dst |= 1ull << qb;
        par ^= ((1ull << qj) - 1) ^ ((1ull << qb) - 1);
        qs[nt++] = qj;
        qs[nt++] = qb;
    }
    std::sort(qs, qs + nt);
    par &= ~(src | dst);
    // constant part: the sign of tau acting on the bare source pattern
    uint64_t x = src;
    int sg = jw_step(x, false, qi);
    if (!single) sg *= jw_step(x, false, qj);
    if (!single) sg *= jw_step(x, true, qb);
    sg *= jw_step(x, true, qa);
    r.src = src;
    r.dst = dst;
    r.par = excitation ? 0ull : par;  // a qubit excitation has no JW string
    for (int t = 0; t < 4; ++t) r.q[t] = t < nt ? (uint32_t)qs[t] : 0u;
    r.nt = nt;
    r.sign0 = excitation ? 1 : sg;
    return r;
}

namespace fsv {

std::vector<uint32_t> strings_of(int M, int N) {
    std::vector<uint32_t> out;
    if (N == 0) {
        out.push_back(0);
        return out;
    }
    if (N > M) return out;
    uint32_t v = (1u << N) - 1;
    const uint32_t lim = 1u << M;
    while (v < lim) {
        out.push_back(v);
        const uint32_t t = v | (v - 1);  // next mask with the same popcount
        v = (t + 1) | (((~t & -~t) - 1) >> (__builtin_ctz(v) + 1));
    }
    return out;
}

uint32_t beta_prefix_parity(int M, int ordering, uint32_t b) {
    auto qubit = [&](int so) { return ordering == 0 ? so : so / 2 + (so % 2) * M; };
    uint32_t pp = 0;
    for (int q = 0; q < M; ++q) {
        int c = 0;
        for (int r = 0; r < M; ++r)
            if ((b >> r & 1u) && qubit(2 * r + 1) < qubit(2 * q)) ++c;
        if (c & 1) pp |= 1u << q;
    }
    return pp;
}

// sign of E_pq = a^+_p a_q acting on string J (q in J, p not in J \ {q})
int sign_epq(uint32_t J, int p, int q) {
    uint64_t x = J;
    int s = jw_step(x, false, q);
    s *= jw_step(x, true, p);
    return s;
}

// Same-spin string Hamiltonian rows by the Slater-Condon rules.  Row I lists
// the diagonal, then the singles (p in I replaced by q not in I), then the
// doubles; the structure does not depend on the integral values.
void build_string_h(int M, const std::vector<uint32_t> &str, const std::vector<int32_t> &rank,
                    const double *ht, const double *g, std::vector<int64_t> &ptr,
                    std::vector<int32_t> &col, std::vector<double> &val) {
    const int M2 = M * M, M3 = M2 * M;
    auto G = [&](int p, int q, int r, int s) { return g[p * M3 + q * M2 + r * M + s]; };
    const size_t ns = str.size();
    ptr.assign(ns + 1, 0);
    col.clear();
    val.clear();
    std::vector<int> occ, vir;
    for (size_t I = 0; I < ns; ++I) {
        const uint32_t s = str[I];
        occ.clear();
        vir.clear();
        for (int p = 0; p < M; ++p) (s >> p & 1u ? occ : vir).push_back(p);
        // diagonal
        double d = 0.0;
        for (int i : occ) d += ht[i * M + i];
        for (int i : occ)
            for (int j : occ) d += 0.5 * (G(i, i, j, j) - G(i, j, j, i));
        col.push_back((int32_t)I);
        val.push_back(d);
        // singles: I = E_pq J with J = I - p + q
        for (int p : occ)
            for (int q : vir) {
                const uint32_t J = (s & ~(1u << p)) | (1u << q);
                double v = ht[p * M + q];
                for (int k : occ)
                    if (k != p) v += G(p, q, k, k) - G(p, k, k, q);
                col.push_back(rank[J]);
                val.push_back(sign_epq(J, p, q) * v);
            }
        // doubles: I = a^+_p a^+_r a_s a_q J, J = I - {p, r} + {q, s}
        for (size_t ip = 0; ip < occ.size(); ++ip)
            for (size_t ir = ip + 1; ir < occ.size(); ++ir)
                for (size_t iq = 0; iq < vir.size(); ++iq)
                    for (size_t is = iq + 1; is < vir.size(); ++is) {
                        const int p = occ[ip], r = occ[ir], q = vir[iq], t = vir[is];
                        const uint32_t J = (s & ~(1u << p) & ~(1u << r)) | (1u << q) | (1u << t);
                        uint64_t x = J;
                        int sg = jw_step(x, false, q);
                        sg *= jw_step(x, false, t);
                        sg *= jw_step(x, true, r);
                        sg *= jw_step(x, true, p);
                        col.push_back(rank[J]);
                        val.push_back(sg * (G(p, q, r, t) - G(p, t, r, q)));
                    }
        ptr[I + 1] = (int64_t)col.size();
    }
}

// One-body part of each entry of build_string_h's rows, in the same order:
// the diagonal entry of row I is sum_{i in I} h_ii (desc = -2 - I), a single
// excitation p <- q is sign * h_pq (desc = p*M+q, bit 30 for a negative sign),
// a double has none (desc = -1).  The rest of each value is two-body only.
void build_string_h_onebody(int M, const std::vector<uint32_t> &str, const std::vector<int32_t> &rank,
                            std::vector<int32_t> &desc) {
    desc.clear();
    std::vector<int> occ, vir;
    for (size_t I = 0; I < str.size(); ++I) {
        const uint32_t s = str[I];
        occ.clear();
        vir.clear();
        for (int p = 0; p < M; ++p) (s >> p & 1u ? occ : vir).push_back(p);
        desc.push_back(-2 - (int32_t)I);
        for (int p : occ)
            for (int q : vir) {
                const uint32_t J = (s & ~(1u << p)) | (1u << q);
                desc.push_back((int32_t)(p * M + q) | (sign_epq(J, p, q) < 0 ? (1 << 30) : 0));
            }
        const size_t nd = occ.size() * (occ.size() - (occ.empty() ? 0 : 1)) / 2 * vir.size() *
                          (vir.size() - (vir.empty() ? 0 : 1)) / 2;
        desc.insert(desc.end(), nd, -1);
    }
    (void)rank;
}

// Gather-form single excitation lists: row I lists (J, p*M+q, sign) with
// E_pq |J> = sign |I>, p in I and q either p or an empty orbital of I.
void build_exc(int M, const std::vector<uint32_t> &str, const std::vector<int32_t> &rank,
               std::vector<uint32_t> &exc, int &nexc) {
    exc.clear();
    nexc = 0;
    for (size_t I = 0; I < str.size(); ++I) {
        const uint32_t s = str[I];
        int cnt = 0;
        // p -> q with q empty first; then the diagonal entries p -> p of the
        // occupied p, the last popcount(s) entries of the list
        for (int p = 0; p < M; ++p) {
            if (!(s >> p & 1u)) continue;
            for (int q = 0; q < M; ++q) {
                if (s >> q & 1u) continue;
                const uint32_t J = (s & ~(1u << p)) | (1u << q);
                exc.push_back(pack_exc((uint32_t)rank[J], (uint32_t)(p * M + q), sign_epq(J, p, q) < 0));
                ++cnt;
            }
        }
        for (int p = 0; p < M; ++p)
            if (s >> p & 1u) {
                exc.push_back(pack_exc((uint32_t)rank[s], (uint32_t)(p * M + p), false));
                ++cnt;
            }
        nexc = cnt;
    }
}

// Per string I: sum over its occupied p of the factor row Lt[pp][0..rp), the
// diagonal entries of I's excitation list folded into one (nstr x rp).
std::vector<double> diag_factor_sums(int M, const std::vector<uint32_t> &str, const std::vector<double> &Lt, int rp) {
    std::vector<double> d(str.size() * (size_t)rp, 0.0);
    for (size_t I = 0; I < str.size(); ++I)
        for (int p = 0; p < M; ++p)
            if (str[I] >> p & 1u)
                for (int l = 0; l < rp; ++l) d[I * rp + l] += Lt[(size_t)(p * M + p) * rp + l];
    return d;
}

void build_bins(int M, const std::vector<uint32_t> &exc, int nexc, std::vector<int32_t> &off,
                std::vector<int32_t> &idx) {
    const int nb = M * M;
    std::vector<std::vector<int32_t>> bins(nb);
    for (size_t k = 0; k < exc.size(); ++k) bins[(exc[k] >> 16) & 0x1FFu].push_back((int32_t)k);
    off.assign(nb + 1, 0);
    idx.clear();
    for (int b = 0; b < nb; ++b) {
        idx.insert(idx.end(), bins[b].begin(), bins[b].end());
        off[b + 1] = (int32_t)idx.size();
    }
    (void)nexc;
}

// The operator compiled for the blocked ordering (qubit p + s*M), whose JW
// basis restricted to the sector is the alpha-first product basis, splits
// into an alpha and a beta part: source/destination/parity bits below M act on
// the alpha string, those above on the beta string.
PairOp build_pair_op(int M, const int32_t *op, const std::vector<uint32_t> &sa,
                     const std::vector<int32_t> &ra, const std::vector<uint32_t> &sb,
                     const std::vector<int32_t> &rb, std::vector<uint32_t> &lists) {
    const RotOp r = compile_op(M, 1, op);
    const uint64_t mask = (1ull << M) - 1ull;
    PairOp o{};
    o.sign0 = r.sign0;
    auto make = [&](uint32_t src, uint32_t dst, uint32_t par, const std::vector<uint32_t> &str,
                    const std::vector<int32_t> &rank, int32_t &n, int64_t &off) {
        if (src == 0 && dst == 0) {  // no part on this spin: the parity mask is empty too
            n = -1;
            off = 0;
            return;
        }
        off = (int64_t)lists.size();
        for (uint32_t s : str) {
            if ((s & src) != src || (s & dst) != 0) continue;
            const uint32_t d = s ^ src ^ dst;
            lists.push_back(pack_pair((uint32_t)rank[s], (uint32_t)rank[d], __builtin_popcount(s & par) & 1));
        }
        n = (int32_t)((int64_t)lists.size() - off);
    };
    make((uint32_t)(r.src & mask), (uint32_t)(r.dst & mask), (uint32_t)(r.par & mask), sa, ra, o.nA, o.offA);
    make((uint32_t)((r.src >> M) & mask), (uint32_t)((r.dst >> M) & mask), (uint32_t)((r.par >> M) & mask),
         sb, rb, o.nB, o.offB);
    return o;
}

// Pair lists of one qubit excitation Q^+_a Q^+_b Q_j Q_i (sign +1 on every
// pair in the plan's qubit basis).  The alpha-first sector basis differs from
// the qubit basis by phi(A, B) = (-1)^N(A, B), N(A, B) = #{(q in A, r in B):
// qubit(r, beta) < qubit(q, alpha)}, so a pair (x, x') carries phi(x) phi(x').
// N is bilinear, hence N(A', B') + N(A, B) = D1(B') + D2(A) mod 2 with
//   D1(B') = sum over the alpha orbitals q the operator changes of
//            #{r in B': qubit(r, beta) < qubit(q, alpha)},
//   D2(A)  = sum over the beta orbitals r it changes of
//            #{q in A: qubit(r, beta) < qubit(q, alpha)},
// an alpha-source factor times a beta-destination factor.  A spin that the
// operator leaves alone gets an explicit diagonal list when its factor is not
// constant (interleaved ordering); in the blocked ordering every factor is 1.
PairOp build_pair_op_qeb(int M, int ordering, const int32_t *op, const std::vector<uint32_t> &sa,
                         const std::vector<int32_t> &ra, const std::vector<uint32_t> &sb,
                         const std::vector<int32_t> &rb, std::vector<uint32_t> &lists) {
    auto qa = [&](int p) { return ordering == 0 ? 2 * p : p; };
    auto qb = [&](int p) { return ordering == 0 ? 2 * p + 1 : p + M; };
    uint32_t ann[2] = {0, 0}, cre[2] = {0, 0};
    for (int t = 2; t < 4; ++t)
        if (op[t] >= 0) ann[op[t] % 2] |= 1u << (op[t] / 2);
    for (int t = 0; t < 2; ++t)
        if (op[t] >= 0) cre[op[t] % 2] |= 1u << (op[t] / 2);
    const uint32_t chA = ann[0] | cre[0], chB = ann[1] | cre[1];
    std::vector<uint32_t> lowB(M, 0), highA(M, 0);  // {r : qb(r) < qa(q)}, {q : qb(r) < qa(q)}
    for (int q = 0; q < M; ++q)
        for (int r = 0; r < M; ++r)
            if (qb(r) < qa(q)) {
                lowB[q] |= 1u << r;
                highA[r] |= 1u << q;
            }
    auto d1 = [&](uint32_t B) {
        int c = 0;
        for (int q = 0; q < M; ++q)
            if (chA >> q & 1u) c += __builtin_popcount(B & lowB[q]);
        return c & 1;
    };
    auto d2 = [&](uint32_t A) {
        int c = 0;
        for (int r = 0; r < M; ++r)
            if (chB >> r & 1u) c += __builtin_popcount(A & highA[r]);
        return c & 1;
    };
    PairOp o{};
    o.sign0 = 1;
    auto part = [&](uint32_t an, uint32_t cr, const std::vector<uint32_t> &str, const std::vector<int32_t> &rank,
                    bool src_factor, int32_t &n, int64_t &off) {
        off = (int64_t)lists.size();
        if (an | cr) {
            for (uint32_t s : str) {
                if ((s & an) != an || (s & cr) != 0) continue;
                const uint32_t d = s ^ an ^ cr;
                lists.push_back(pack_pair((uint32_t)rank[s], (uint32_t)rank[d], src_factor ? d2(s) : d1(d)));
            }
        } else {
            bool any = false;
            for (uint32_t s : str) any = any || (src_factor ? d2(s) : d1(s));
            if (!any) {
                n = -1;
                off = 0;
                return;
            }
            for (uint32_t s : str)
                lists.push_back(pack_pair((uint32_t)rank[s], (uint32_t)rank[s], src_factor ? d2(s) : d1(s)));
        }
        n = (int32_t)((int64_t)lists.size() - off);
    };
    part(ann[0], cre[0], sa, ra, true, o.nA, o.offA);
    part(ann[1], cre[1], sb, rb, false, o.nB, o.offB);
    return o;
}

// Pivoted Cholesky of a symmetric positive semidefinite n x n matrix G: the
// largest remaining diagonal is taken as the next pivot until every residual
// diagonal is below tol * max(diag).  Returns the rank R (L holds R rows of
// length n, G ~ sum_k L_k L_k^T) or -1 when G is not positive semidefinite
// within that tolerance.
int pivoted_cholesky(int n, const double *G, double tol, std::vector<double> &L) {
    std::vector<double> d(n);
    double dmax = 0.0;
    for (int i = 0; i < n; ++i) {
        d[i] = G[(size_t)i * n + i];
        dmax = std::max(dmax, d[i]);
    }
    L.clear();
    if (dmax <= 0.0) return 0;
    const double cut = tol * dmax;
    int R = 0;
    while (R < n) {
        int p = 0;
        for (int i = 1; i < n; ++i)
            if (d[i] > d[p]) p = i;
        if (d[p] <= cut) break;
        const double piv = std::sqrt(d[p]);
        std::vector<double> ell(n);
        for (int i = 0; i < n; ++i) {
            double v = G[(size_t)i * n + p];
            for (int k = 0; k < R; ++k) v -= L[(size_t)k * n + i] * L[(size_t)k * n + p];
            ell[i] = v / piv;
        }
        for (int i = 0; i < n; ++i) d[i] -= ell[i] * ell[i];
        L.insert(L.end(), ell.begin(), ell.end());
        ++R;
    }
    for (int i = 0; i < n; ++i)
        if (d[i] < -cut) return -1;
    return R;
}

}  // namespace fsv

namespace {

// Choose the factorised alpha-beta product when (pq|rs) has a small exact
// pivoted-Cholesky rank: per sector element it costs R (e_a + e_b) instead of
// e_a e_b multiply-adds.  The factorisation must reproduce g to 1e-12 relative.
int lr_pad(int) { return 8; }  // factor columns of the factorised kernels (ranks <= 8)

void choose_sigma(fsv_plan &P, int &R_out, std::vector<double> &Lt_out) {
    R_out = 0;
    const char *mode = std::getenv("FSV_SIGMA");
    if (mode && std::strcmp(mode, "direct") == 0) return;
    const int M2 = P.M * P.M;
    if (P.nexcA <= 0 || P.nexcB <= 0 || M2 > 511) return;
    std::vector<double> L;
    const int R = pivoted_cholesky(M2, P.g.data(), 1e-14, L);
    // ranks above 8 take the direct product: the 16- and 32-column factorised
    // kernels are kept out of use (no parity test of theirs has passed)
    if (R <= 0 || R > 8) return;
    double gmax = 0.0, err = 0.0;
    for (int i = 0; i < M2; ++i)
        for (int j = 0; j < M2; ++j) {
            double v = 0.0;
            for (int k = 0; k < R; ++k) v += L[(size_t)k * M2 + i] * L[(size_t)k * M2 + j];
            gmax = std::max(gmax, std::fabs(P.g[(size_t)i * M2 + j]));
            err = std::max(err, std::fabs(v - P.g[(size_t)i * M2 + j]));
        }
    if (err > 1e-12 * std::max(1.0, gmax)) return;
    const bool forced = mode && std::strcmp(mode, "lowrank") == 0;
    if (!forced && (int64_t)R * (P.nexcA + P.nexcB) >= (int64_t)P.nexcA * P.nexcB) return;
    // the beta step stages one row of the intermediate (complex for the dense
    // engine) with one factor column in LDS
    const int rp = lr_pad(R);
    if (P.nsb * 16 + (int64_t)M2 * 8 > 163840) return;
    R_out = R;
    Lt_out.assign((size_t)M2 * rp, 0.0);  // M^2 x rp, zero beyond column R
    for (int k = 0; k < R; ++k)
        for (int i = 0; i < M2; ++i) Lt_out[(size_t)i * rp + k] = L[(size_t)k * M2 + i];
}

// Dense copies of the same-spin string Hamiltonians, rebuilt on the device
// from the CSR rows whenever the one-body part changes.
int refresh_dense_same_spin(fsv_plan &P) {
    if (!P.d_ha_dense) return FSV_OK;
    HIPCHECK(launch_csr_dense(P.d_ha_ptr, P.d_ha_col, P.d_ha_val, P.d_ha_dense, P.nsa, P.work));
    HIPCHECK(launch_csr_dense(P.d_hb_ptr, P.d_hb_col, P.d_hb_val, P.d_hb_dense, P.nsb, P.work));
    HIPCHECK(launch_ctranspose(false, P.d_hb_dense, P.d_hb_dense_t, P.nsb, P.nsb, P.work));
    HIPCHECK(hipStreamSynchronize(P.work));
    return FSV_OK;
}

// Same-spin products as dense FP64 GEMMs when the string Hamiltonian is
// dense enough that the matrix cores beat gathering its rows: per output
// element a sparse row costs nnz 8-byte gathers at ~10 TB/s, a dense row
// 2 nsa flops at ~40 TFLOP/s (FSV_SAME_SPIN = dense | sparse overrides).
bool want_dense_same_spin(const fsv_plan &P) {
    const char *m = std::getenv("FSV_SAME_SPIN");
    if (m && std::strcmp(m, "sparse") == 0) return false;
    const double bytes = 8.0 * ((double)P.nsa * P.nsa + (double)P.nsb * P.nsb);
    if (bytes > 16e9) return false;
    if (m && std::strcmp(m, "dense") == 0) return true;
    if (P.nsa * P.nsb < 4096) return false;
    const double nnz_a = (double)P.ha_col.size() / (double)P.nsa, nnz_b = (double)P.hb_col.size() / (double)P.nsb;
    return nnz_a * 16.0 > (double)P.nsa && nnz_b * 16.0 > (double)P.nsb;
}

// New one-body potential: h + v goes up (M^2 doubles) and the string
// Hamiltonian values (and their dense copies) are rebuilt on the device from
// the fixed two-body parts and the one-body descriptors.
int upload_hamiltonian_values(fsv_plan &P) {
    std::vector<double> ht(P.h);
    for (size_t i = 0; i < ht.size(); ++i) ht[i] += P.v[i];
    // earlier work on the stream (a previous refresh reading h + v, or
    // products using the old values) completes before h + v is overwritten
    HIPCHECK(hipStreamSynchronize(P.work));
    int rc;
    if ((rc = upload(P, P.d_htilde, ht.data(), ht.size()))) return rc;
    HIPCHECK(launch_string_h_values(P.d_ha_val, P.d_ha_v2, P.d_ha_desc, P.d_str_a, P.d_htilde, P.M,
                                    (int64_t)P.ha_col.size(), P.work));
    HIPCHECK(launch_string_h_values(P.d_hb_val, P.d_hb_v2, P.d_hb_desc, P.d_str_b, P.d_htilde, P.M,
                                    (int64_t)P.hb_col.size(), P.work));
    if (P.d_ha_dense) {
        HIPCHECK(launch_csr_dense(P.d_ha_ptr, P.d_ha_col, P.d_ha_val, P.d_ha_dense, P.nsa, P.work));
        HIPCHECK(launch_csr_dense(P.d_hb_ptr, P.d_hb_col, P.d_hb_val, P.d_hb_dense, P.nsb, P.work));
        HIPCHECK(launch_ctranspose(false, P.d_hb_dense, P.d_hb_dense_t, P.nsb, P.nsb, P.work));
    }
    return FSV_OK;
}

// Byte model of one pair kernel (read + write of the touched 128-byte lines).
double op_line_bytes(const fsv_plan &P, const RotOp &r) {
    const int low = P.amp_bytes == 16 ? 3 : 4;
    int hi = 0;
    for (int t = 0; t < r.nt; ++t) hi += (int)r.q[t] >= low;
    const double full = 2.0 * std::ldexp(1.0, P.n) * P.amp_bytes;
    const double frac = hi == 0 ? 1.0 : std::min(1.0, std::ldexp(1.0, 1 - hi));
    return full * frac;
}

void plan_segments(fsv_plan &P) {
    P.segs.clear();
    P.tile_bits = P.precision == 0 ? 12 : 13;
    const bool allow = P.n > P.tile_bits && std::getenv("FSV_NO_FUSE") == nullptr;
    const bool force = std::getenv("FSV_FORCE_FUSE") != nullptr;
    const double full = 2.0 * std::ldexp(1.0, P.n) * P.amp_bytes;
    int k = 0;
    while (k < P.K) {
        int e = k;
        double cost = 0.0;
        if (allow) {
            while (e < P.K && e - k < max_fused_run()) {
                const RotOp &r = P.rot[e];
                if ((int)r.q[r.nt - 1] >= P.tile_bits) break;
                cost += op_line_bytes(P, r);
                ++e;
            }
        }
        if (e - k >= 2 && (force || full < 0.9 * cost)) {
            P.segs.push_back({k, e, true});
            k = e;
        } else {
            P.segs.push_back({k, k + 1, false});
            ++k;
        }
    }
}

int upload_counts(fsv_plan &P) {
    std::vector<int> gc(std::max(P.K, 1), 0);
    for (int k = 0; k < P.K; ++k) gc[k] = (int)rot_grid(P.npairs[k], P.shape_adj);
    // operators of a fused run: one partial per workgroup of the fused adjoint
    for (const auto &sg : P.segs)
        if (sg.fused)
            for (int k = sg.k0; k < sg.k1; ++k) gc[k] = (int)fused_grid(1ull << P.n, P.tile_bits);
    return upload(P, P.d_gcount, gc.data(), (size_t)P.K);
}

void drop_graphs(fsv_plan &P) {
    ++P.gen;  // graphs of pools built on this plan are stale too
    if (P.g_eg) (void)hipGraphExecDestroy(P.g_eg);
    if (P.g_e) (void)hipGraphExecDestroy(P.g_e);
    P.g_eg = nullptr;
    P.g_e = nullptr;
    P.g_eg_psi = P.g_eg_lam = P.g_e_psi = nullptr;
}

// The plan's stream waits for the work queued on the caller's stream.  Calls
// that wait for their own work on the host before returning first ask
// whether the caller's stream is idle, in which case there is nothing to
// wait for (an event record and a stream wait cost ~15 us of host time, a
// query of an idle stream well under 1 us).  The stage calls fence
// unconditionally: after the previous stage call's fence_out the caller's
// stream is still waiting, so the query would only add its own cost.
int fence_in(fsv_plan &P, bool skip_if_idle = false) {
    if (skip_if_idle && stream_idle(P.user)) return FSV_OK;
    HIPCHECK(hipEventRecord(P.ev_in, P.user));
    HIPCHECK(hipStreamWaitEvent(P.work, P.ev_in, 0));
    return FSV_OK;
}

// Later work on the caller's stream waits for the plan's.  Calls that have
// waited for their work on the host end without it: nothing queued later
// can overtake work that has completed.
int fence_out(fsv_plan &P) {
    HIPCHECK(hipEventRecord(P.ev_out, P.work));
    HIPCHECK(hipStreamWaitEvent(P.user, P.ev_out, 0));
    return FSV_OK;
}

// ---- enqueue helpers (no synchronisation; usable under stream capture) ----
int enq_forward_dense(fsv_plan &P, void *psi) {
    HIPCHECK(launch_fill_zero(psi, ((size_t)1 << P.n) * P.amp_bytes, P.work));
    if (P.n_init)
        HIPCHECK(launch_set_list(psi, P.precision == 0 ? V_C128 : V_C64, P.d_init_didx, P.d_init_dval, P.n_init,
                                 P.work));
    else
        HIPCHECK(launch_set_amp(psi, P.precision == 0 ? V_C128 : V_C64, P.ref_index, 1.0, P.work));
    for (const auto &sg : P.segs) {
        if (sg.fused) {
            HIPCHECK(launch_rot_fused(P.precision, psi, P.d_rot, P.d_cs, sg.k0, sg.k1, P.tile_bits,
                                      1ull << P.n, P.work));
        } else {
            const int k = sg.k0;
            HIPCHECK(launch_rot(P.precision, P.wide, psi, P.rot[k], P.d_cs, k, P.npairs[k],
                                P.shape_rot, P.work));
        }
    }
    return FSV_OK;
}

// S = H C on the sector (alpha-first basis, complex or real FP64) and
// E = Re<C|S> into d_out[0].
int enq_sector_sigma(fsv_plan &P, bool cplex, const void *C, void *S) {
    bool zipped = false;
    HIPCHECK(launch_sector_sigma(cplex, P.tabs, C, S, P.d_CT, P.d_ST, P.d_epart, P.work,
                                 P.zip_in_sigma && !cplex ? (void *)P.d_C : nullptr, &zipped));
    P.z_ready = zipped;
    if (!P.defer_e) HIPCHECK(launch_reduce_rows(P.d_epart, P.d_ecount, 0, 1, 1.0, P.d_out, P.work));
    return FSV_OK;
}

// Dense input: gather the complex sector, H on it; lam == nullptr: energy only.
int enq_sigma_dense(fsv_plan &P, const void *psi, void *lam) {
    HIPCHECK(launch_gather(P.precision, psi, P.d_Xa, P.d_Xb, P.d_sa, P.d_PPb, P.nsa, P.nsb, P.d_C, P.work));
    int rc = enq_sector_sigma(P, true, P.d_C, P.d_S);
    if (rc) return rc;
    if (lam) {
        HIPCHECK(launch_fill_zero(lam, ((size_t)1 << P.n) * P.amp_bytes, P.work));
        HIPCHECK(launch_scatter(P.precision, lam, P.d_S, P.d_Xa, P.d_Xb, P.d_sa, P.d_PPb, P.nsa, P.nsb, P.work));
    }
    return FSV_OK;
}

int enq_reverse_dense(fsv_plan &P, void *psi, void *lam) {
    const int G = max_grid();
    for (auto it = P.segs.rbegin(); it != P.segs.rend(); ++it) {
        if (it->fused) {
            HIPCHECK(launch_adj_fused(P.precision, psi, lam, P.d_rot, P.d_cs, it->k0, it->k1, P.tile_bits,
                                      1ull << P.n, P.d_gpart, G, P.work));
            continue;
        }
        for (int k = it->k1 - 1; k >= it->k0; --k)
            HIPCHECK(launch_adj(P.precision, P.wide, psi, lam, P.rot[k], P.d_cs, k, P.npairs[k],
                                P.shape_adj, P.d_gpart + (size_t)k * G, P.work));
    }
    if (P.defer_e)
        HIPCHECK(launch_reduce_eg(P.d_epart, P.d_ecount, P.d_gpart, P.d_gcount, G, P.K, P.d_out, P.work));
    else
        HIPCHECK(launch_reduce_rows(P.d_gpart, P.d_gcount, G, P.K, 2.0, P.d_out + 1, P.work));
    return FSV_OK;
}

// One group of the forward sweep: a fused run in one launch, or its single
// operator.  t0, t1 (optional, profiling): a packet run's kernel start and end
// times, or events recorded before and after the group's launches.
int enq_group_fwd(fsv_plan &P, void *c, const FGroup &g, hipEvent_t t0 = nullptr, hipEvent_t t1 = nullptr) {
    if (g.fused == 2) {
        HIPCHECK(launch_packets(P.svt, false, c, P.ffwd, g, P.d_cs, nullptr, 0, P.work, t0, t1));
        return FSV_OK;
    }
    if (t0) HIPCHECK(hipEventRecord(t0, P.work));
    if (g.fused) {
        HIPCHECK(launch_fused(P.svt, false, c, nullptr, P.ffwd, g, P.d_pops, P.d_cs, P.nsb, nullptr, 0, P.work));
    } else {
        for (int k = g.k0; k < g.k0 + g.nops; ++k)
            HIPCHECK(launch_crot(P.svt, c, P.pops[k], P.d_plists, P.d_cs, k, P.nsa, P.nsb, P.work));
    }
    if (t1) HIPCHECK(hipEventRecord(t1, P.work));
    return FSV_OK;
}

// One group of the adjoint sweep (operators last to first).  Packet
// schedules run on the interleaved pairs z in d_C (c and lam_c are unused).
// The adjoint sweep runs on interleaved (psi, lam) pairs in the sector
// workspace unless one of its runs is an LDS-tile run (those read the two
// arrays): one 16-byte access per amplitude touches fewer cache lines than two
// 8-byte accesses to separate arrays (at 30 qubits, 11 % fewer bytes of lines
// for the per-operator adjoint steps, whose pairs are scattered within rows).
bool reverse_on_pairs(const fsv_plan &P) {
    if (P.frev.packets) return true;
    for (const FGroup &g : P.frev.groups)
        if (g.fused) return false;
    return true;
}

int enq_group_rev(fsv_plan &P, void *c, void *lam_c, const FGroup &g, hipEvent_t t0 = nullptr,
                  hipEvent_t t1 = nullptr, bool store = true) {
    const int G = max_grid();
    if (reverse_on_pairs(P)) {
        void *z = P.d_C;
        if (g.fused) {
            HIPCHECK(launch_packets(P.svt, true, z, P.frev, g, P.d_cs, P.d_gpart, G, P.work, t0, t1, store));
            return FSV_OK;
        }
        if (t0) HIPCHECK(hipEventRecord(t0, P.work));
        for (int k = g.k0 + g.nops - 1; k >= g.k0; --k)
            HIPCHECK(launch_cadj_zip(P.svt, z, P.pops[k], P.d_plists, P.d_cs, k, P.nsa, P.nsb,
                                     P.d_gpart + (size_t)k * G, P.work));
        if (t1) HIPCHECK(hipEventRecord(t1, P.work));
        return FSV_OK;
    }
    if (t0) HIPCHECK(hipEventRecord(t0, P.work));
    if (g.fused) {
        HIPCHECK(launch_fused(P.svt, true, c, lam_c, P.frev, g, P.d_pops, P.d_cs, P.nsb, P.d_gpart, G, P.work));
    } else {
        for (int k = g.k0 + g.nops - 1; k >= g.k0; --k)
            HIPCHECK(launch_cadj(P.svt, c, lam_c, P.pops[k], P.d_plists, P.d_cs, k, P.nsa, P.nsb,
                                 P.d_gpart + (size_t)k * G, P.work));
    }
    if (t1) HIPCHECK(hipEventRecord(t1, P.work));
    return FSV_OK;
}

// ---- sector-compressed engine: the state is C[Ia][Ib] in the first
// nsa*nsb amplitudes of the caller's buffer.  With real angles and real
// integrals every amplitude stays real, so it is stored real (FP64 or FP32). ----
// From the reference state the forward sweep's first runs act on a state
// that is zero outside a few components: every other packet maps zeros to
// zeros, so only the packets the plan recorded as holding nonzero amplitudes
// are launched (FGroup::sub_n; none when the run leaves the support alone).
// Not for a multi-determinant start.
FGroup forward_run(const fsv_plan &P, const FGroup &g) {
    FGroup h = g;
    if (P.n_init || g.fused != 2 || g.sub_n < 0) return h;
    h.ent_off = g.sub_ent_off;
    h.reg_off = g.sub_reg_off;
    h.n_packets = g.sub_n;
    return h;
}

int enq_forward_sector(fsv_plan &P, void *c) {
    HIPCHECK(launch_fill_zero(c, (size_t)P.dim * vtype_bytes(P.svt), P.work));
    // The reference is string 0 x string 0.  Its alpha-first amplitude carries
    // the ordering sign so that the dense image starts at exactly +1 |ref>.
    if (P.n_init)
        HIPCHECK(launch_set_list(c, P.svt, P.d_init_sidx, P.d_init_sval, P.n_init, P.work));
    else
        HIPCHECK(launch_set_amp(c, P.svt, 0, P.ref_phase, P.work));
    for (const FGroup &g : P.ffwd.groups) {
        const int rc = enq_group_fwd(P, c, forward_run(P, g));
        if (rc) return rc;
    }
    return FSV_OK;
}

// lam_c == nullptr: energy only.  FP32 states are widened for the product.
int enq_sigma_sector(fsv_plan &P, const void *c, void *lam_c) {
    if (P.svt == V_F64) return enq_sector_sigma(P, false, c, lam_c ? lam_c : (void *)P.d_S);
    HIPCHECK(launch_convert(V_F32, c, V_F64, P.d_C, P.dim, P.work));
    int rc = enq_sector_sigma(P, false, P.d_C, P.d_S);
    if (rc) return rc;
    if (lam_c) HIPCHECK(launch_convert(V_F64, P.d_S, V_F32, lam_c, P.dim, P.work));
    return FSV_OK;
}

// Packet schedules first interleave psi and lam into d_C (2 dim values of
// the state's type, within its dim double2), so that each gather of the packet
// kernels moves both; psi and lam are then left as they were.  Other
// schedules un-rotate c and lam_c in place.
int enq_reverse_sector(fsv_plan &P, void *c, void *lam_c) {
    const int G = max_grid();
    if (reverse_on_pairs(P) && !P.z_ready) HIPCHECK(launch_zip(P.svt, c, lam_c, P.d_C, P.dim, P.work));
    P.z_ready = false;
    for (auto it = P.frev.groups.rbegin(); it != P.frev.groups.rend(); ++it) {
        // the sweep's last run: its un-rotated psi and lam are not needed
        const int rc = enq_group_rev(P, c, lam_c, *it, nullptr, nullptr, std::next(it) != P.frev.groups.rend());
        if (rc) return rc;
    }
    if (P.defer_e)
        HIPCHECK(launch_reduce_eg(P.d_epart, P.d_ecount, P.d_gpart, P.d_ccount, G, P.K, P.d_out, P.work));
    else
        HIPCHECK(launch_reduce_rows(P.d_gpart, P.d_ccount, G, P.K, 2.0, P.d_out + 1, P.work));
    return FSV_OK;
}

// The forward (adjoint = 0: initial state, then the groups) or adjoint sweep
// (adjoint = 1: groups last to first on psi, lam, then the gradient reduction)
// launched eagerly; ms[i] = time of group i (operator order): a packet run's
// kernel time (events that take its start and end), the time between events
// around the launches of any other group.  Synchronises the work stream.
int time_sweep_sector(fsv_plan &P, int adjoint, void *c, void *lam_c, float *ms) {
    const FusedSched &S = adjoint ? P.frev : P.ffwd;
    const int n = (int)S.groups.size();
    std::vector<hipEvent_t> ev(2 * (size_t)n, nullptr);  // group i: ev[2 i], ev[2 i + 1]
    int rc = FSV_OK;
    for (auto &e : ev)
        if (!rc && hipEventCreate(&e) != hipSuccess) rc = fail(FSV_EDEVICE, "hipEventCreate failed");
    if (!rc && !adjoint) {
        if (hipSuccess != launch_fill_zero(c, (size_t)P.dim * vtype_bytes(P.svt), P.work))
            rc = fail(FSV_EDEVICE, "fill launch failed");
        else if (P.n_init && hipSuccess != launch_set_list(c, P.svt, P.d_init_sidx, P.d_init_sval, P.n_init, P.work))
            rc = fail(FSV_EDEVICE, "initial-state launch failed");
        else if (!P.n_init && hipSuccess != launch_set_amp(c, P.svt, 0, P.ref_phase, P.work))
            rc = fail(FSV_EDEVICE, "initial-state launch failed");
    }
    if (!rc && adjoint && reverse_on_pairs(P) && hipSuccess != launch_zip(P.svt, c, lam_c, P.d_C, P.dim, P.work))
        rc = fail(FSV_EDEVICE, "interleave launch failed");
    for (int t = 0; t < n && !rc; ++t) {
        const int i = adjoint ? n - 1 - t : t;
        hipEvent_t t0 = ev[2 * (size_t)i], t1 = ev[2 * (size_t)i + 1];
        rc = adjoint ? enq_group_rev(P, c, lam_c, S.groups[i], t0, t1)
                     : enq_group_fwd(P, c, forward_run(P, S.groups[i]), t0, t1);
    }
    if (!rc && adjoint &&
        hipSuccess != launch_reduce_rows(P.d_gpart, P.d_ccount, max_grid(), P.K, 2.0, P.d_out + 1, P.work))
        rc = fail(FSV_EDEVICE, "reduction launch failed");
    if (!rc && hipStreamSynchronize(P.work) != hipSuccess) rc = fail(FSV_EDEVICE, "stream synchronize failed");
    for (int i = 0; i < n && !rc; ++i) {
        float v = 0.f;
        if (hipEventElapsedTime(&v, ev[2 * (size_t)i], ev[2 * (size_t)i + 1]) != hipSuccess)
            rc = fail(FSV_EDEVICE, "event timing failed");
        ms[i] = v;
    }
    for (auto &e : ev)
        if (e) (void)hipEventDestroy(e);
    return rc;
}

int enq_forward(fsv_plan &P, void *psi) {
    return P.engine == 0 ? enq_forward_sector(P, psi) : enq_forward_dense(P, psi);
}

int enq_sigma(fsv_plan &P, const void *psi, void *lam) {
    return P.engine == 0 ? enq_sigma_sector(P, psi, lam) : enq_sigma_dense(P, psi, lam);
}

int enq_reverse(fsv_plan &P, void *psi, void *lam) {
    return P.engine == 0 ? enq_reverse_sector(P, psi, lam) : enq_reverse_dense(P, psi, lam);
}

// Dense output of the ansatz: prepared on the sector in the workspace, then
// expanded (zero elsewhere) into the caller's 2^n buffer.
int enq_ansatz_dense_out(fsv_plan &P, void *psi) {
    if (P.engine != 0) return enq_forward_dense(P, psi);
    int rc = enq_forward_sector(P, P.d_S);
    if (rc) return rc;
    const double *S = (const double *)P.d_S;
    if (P.svt == V_F32) {
        HIPCHECK(launch_convert(V_F32, P.d_S, V_F64, P.d_C, P.dim, P.work));
        S = (const double *)P.d_C;
    }
    HIPCHECK(launch_fill_zero(psi, ((size_t)1 << P.n) * P.amp_bytes, P.work));
    HIPCHECK(launch_scatter_real(P.precision, psi, S, P.d_Xa, P.d_Xb, P.d_sa, P.d_PPb, P.nsa, P.nsb, P.work));
    return FSV_OK;
}

int upload_theta(fsv_plan &P, const double *theta) {
    if (P.K > 0 && !theta) return fail(FSV_EINVAL, "theta is NULL");
    if (!finite_all(theta, (size_t)P.K)) return fail(FSV_ENONFINITE, "non-finite theta");
    double *h = P.h_pin;
    if (P.cs_pending) {  // the previous upload may still be reading h
        HIPCHECK(hipEventSynchronize(P.ev_cs));
        P.cs_pending = false;
    }
    for (int k = 0; k < P.K; ++k) {
        h[2 * k] = std::cos(theta[k]);
        h[2 * k + 1] = std::sin(theta[k]);
    }
    if (P.K > 0) {
        HIPCHECK(hipMemcpyAsync(P.d_cs, h, sizeof(double) * 2 * P.K, hipMemcpyHostToDevice, P.work));
        HIPCHECK(hipEventRecord(P.ev_cs, P.work));
        P.cs_pending = true;
    }
    return FSV_OK;
}

// energy_grad's angles: cos / sin into the coherent pinned block that the
// graph's first node copies to the device (no separate copy call).
int stage_theta(fsv_plan &P, const double *theta) {
    if (P.K > 0 && !theta) return fail(FSV_EINVAL, "theta is NULL");
    if (!finite_all(theta, (size_t)P.K)) return fail(FSV_ENONFINITE, "non-finite theta");
    for (int k = 0; k < P.K; ++k) {
        P.h_cs[2 * k] = std::cos(theta[k]);
        P.h_cs[2 * k + 1] = std::sin(theta[k]);
    }
    return FSV_OK;
}

int download_out(fsv_plan &P, double *E_out, double *grad_out, bool with_grad) {
    double *h = P.h_pin + 2 * (size_t)P.K;
    const size_t cnt = with_grad ? (size_t)P.K + 1 : 1;
    HIPCHECK(hipMemcpyAsync(h, P.d_out, sizeof(double) * cnt, hipMemcpyDeviceToHost, P.work));
    HIPCHECK(hipStreamSynchronize(P.work));
    if (E_out) *E_out = h[0];
    if (with_grad && grad_out) std::memcpy(grad_out, h + 1, sizeof(double) * P.K);
    return FSV_OK;
}

typedef int (*enq_fn)(fsv_plan &, void *, void *);

// The energy's partial sums wait for the gradients' reduction (one launch
// for both, the same ordered sums).
int run_energy_grad_body(fsv_plan &P, void *psi, void *lam) {
    int rc;
    if ((rc = enq_forward(P, psi))) return rc;
    P.defer_e = true;
    P.zip_in_sigma = P.engine == 0 && P.svt == V_F64 && reverse_on_pairs(P);
    if (!(rc = enq_sigma(P, psi, lam))) rc = enq_reverse(P, psi, lam);
    P.defer_e = false;
    P.zip_in_sigma = P.z_ready = false;
    return rc;
}

int run_energy_body(fsv_plan &P, void *psi) {
    int rc;
    if ((rc = enq_forward(P, psi))) return rc;
    if ((rc = enq_sigma(P, psi, nullptr))) return rc;
    return FSV_OK;
}

// Capture body into a graph exec; false when capture is unavailable.
template <typename F>
int capture(fsv_plan &P, F body, hipGraphExec_t *exec) {
    hipGraph_t graph = nullptr;
    HIPCHECK(hipStreamBeginCapture(P.work, hipStreamCaptureModeThreadLocal));
    int rc = body();
    hipGraph_t g2 = nullptr;
    hipError_t e = hipStreamEndCapture(P.work, &g2);
    graph = g2;
    if (rc) {
        if (graph) (void)hipGraphDestroy(graph);
        return rc;
    }
    if (e != hipSuccess) return fail(FSV_EDEVICE, "hipStreamEndCapture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(FSV_EDEVICE, "hipGraphInstantiate: %s", hipGetErrorString(e));
    return FSV_OK;
}

int launch_energy_grad(fsv_plan &P, void *psi, void *lam) {
    if (!P.use_graph) {
        HIPCHECK(launch_copy_doubles(P.h_cs, P.d_cs, 2 * P.K, P.work));
        return run_energy_grad_body(P, psi, lam);
    }
    if (!P.g_eg || P.g_eg_psi != psi || P.g_eg_lam != lam) {
        if (P.g_eg) (void)hipGraphExecDestroy(P.g_eg);
        P.g_eg = nullptr;
        int rc = capture(P, [&]() {
            HIPCHECK(launch_copy_doubles(P.h_cs, P.d_cs, 2 * P.K, P.work));
            return run_energy_grad_body(P, psi, lam);
        }, &P.g_eg);
        if (rc) {
            P.g_eg = nullptr;
            return rc;
        }
        P.g_eg_psi = psi;
        P.g_eg_lam = lam;
    }
    HIPCHECK(hipGraphLaunch(P.g_eg, P.work));
    return FSV_OK;
}

int launch_energy_only(fsv_plan &P, void *psi) {
    if (!P.use_graph) return run_energy_body(P, psi);
    if (!P.g_e || P.g_e_psi != psi) {
        if (P.g_e) (void)hipGraphExecDestroy(P.g_e);
        P.g_e = nullptr;
        int rc = capture(P, [&]() { return run_energy_body(P, psi); }, &P.g_e);
        if (rc) {
            P.g_e = nullptr;
            return rc;
        }
        P.g_e_psi = psi;
    }
    HIPCHECK(hipGraphLaunch(P.g_e, P.work));
    return FSV_OK;
}

// Fused runs of both sweeps for the current LDS budgets, and the gradient
// partial counts of the adjoint sweep that they imply.
int rebuild_fused(fsv_plan &P) {
    FusedOpts o;
    o.es = vtype_bytes(P.svt);
    o.mode = P.fuse_mode;
    o.max_tiles = max_grid();
    const size_t lim = fused_lds_limit();
    o.lds_limit = lim;
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && cus > 0)
        o.cus = cus;
    (void)hipGetLastError();
    int rc;
    if (P.fuse_mode == 3 && P.dim <= packet_max_dim()) {
        // both sweeps run the same packet runs; above the default size (only
        // on request) every run is one: the cost model's rates are those of
        // cache-resident states, and at 30 qubits every run pays
        o.mode = P.dim <= packet_default_dim() ? 0 : 2;
        o.arrays = 2;
        if ((rc = build_packets(P.nsa, P.nsb, P.pops, P.h_plists, o, P.frev))) return rc;
        P.ffwd.share(P.frev);
    } else {
        if (o.mode == 3) o.mode = 0;
        o.arrays = 1;
        o.budget = std::min(P.fuse_budget_fwd, lim);
        if ((rc = build_fused(P.M, P.sa, P.sb, P.pops, P.h_plists, P.ops, o, P.ffwd))) return rc;
        o.arrays = 2;
        o.budget = std::min(P.fuse_budget_rev, lim);
        if ((rc = build_fused(P.M, P.sa, P.sb, P.pops, P.h_plists, P.ops, o, P.frev))) return rc;
    }
    std::vector<int> ccount(std::max(P.K, 1), 0);
    for (int k = 0; k < P.K; ++k)
        ccount[k] = P.frev.count[k] >= 0 ? P.frev.count[k] : cadj_blocks(P.pops[k], P.nsa, P.nsb);
    drop_graphs(P);
    return upload(P, P.d_ccount, ccount.data(), (size_t)P.K);
}

// Bounds of the host tables before they go to the device, as the kernels read
// them: pair-list entries (15-bit string ranks) name strings of their spin,
// excitation words (16-bit rank, 9-bit orbital pair) name strings and orbital
// pairs, each string's list ends with its diagonal excitations, the bins and
// the CSR string Hamiltonians index inside their arrays, and every gradient
// partial count fits the partial rows.
int check_tables(const fsv_plan &P, const std::vector<uint32_t> &excA, const std::vector<uint32_t> &excB,
                 const std::vector<int32_t> &boA, const std::vector<int32_t> &biA, const std::vector<int32_t> &boB,
                 const std::vector<int32_t> &biB) {
    const int M = P.M, M2 = M * M;
    if (P.nsa > 32768 || P.nsb > 32768 || M2 > 511) return fail(FSV_EINVAL, "internal: sector too large for the tables");
    for (int k = 0; k < P.K; ++k) {
        const PairOp &o = P.pops[k];
        auto side = [&](int32_t n, int64_t off, int64_t ns) {
            if (n < -1 || (n >= 0 && off + n > (int64_t)P.h_plists.size())) return false;
            for (int32_t u = 0; u < n; ++u) {
                const uint32_t e = P.h_plists[off + u];
                if ((int64_t)(e & 0x7FFFu) >= ns || (int64_t)((e >> 15) & 0x7FFFu) >= ns) return false;
            }
            return true;
        };
        if (!side(o.nA, o.offA, P.nsa) || !side(o.nB, o.offB, P.nsb))
            return fail(FSV_EINVAL, "internal: pair list of operator %d out of range", k);
    }
    auto exc_ok = [&](const std::vector<uint32_t> &exc, int nexc, int64_t ns, int nd) {
        if ((int64_t)exc.size() != ns * nexc || nd > nexc) return false;
        for (int64_t I = 0; I < ns; ++I)
            for (int e = 0; e < nexc; ++e) {
                const uint32_t w = exc[(size_t)I * nexc + e];
                const uint32_t pq = (w >> 16) & 0x1FFu;
                if ((int64_t)(w & 0xFFFFu) >= ns || (int)pq >= M2) return false;
                if (e >= nexc - nd && ((w & 0xFFFFu) != (uint32_t)I || pq % (M + 1) != 0)) return false;
            }
        return true;
    };
    if (!exc_ok(excA, P.nexcA, P.nsa, P.na) || !exc_ok(excB, P.nexcB, P.nsb, P.nb))
        return fail(FSV_EINVAL, "internal: excitation lists out of range");
    auto bins_ok = [&](const std::vector<int32_t> &off, const std::vector<int32_t> &idx, size_t n) {
        if ((int)off.size() != M2 + 1 || off[0] != 0 || (size_t)off[M2] != idx.size() || idx.size() != n) return false;
        for (int b = 0; b < M2; ++b)
            if (off[b + 1] < off[b]) return false;
        for (int32_t i : idx)
            if (i < 0 || (size_t)i >= n) return false;
        return true;
    };
    if (!bins_ok(boA, biA, excA.size()) || !bins_ok(boB, biB, excB.size()))
        return fail(FSV_EINVAL, "internal: density-matrix bins out of range");
    for (int k = 0; k < P.K; ++k)
        if (P.frev.count[k] > max_grid()) return fail(FSV_EINVAL, "internal: gradient partials of operator %d", k);
    if (P.pin_doubles < 3 * (size_t)P.K + 1 + 4 * (size_t)M2) return fail(FSV_EINVAL, "internal: pinned buffer");
    return FSV_OK;
}

int check_csr(const std::vector<int64_t> &ptr, const std::vector<int32_t> &col, size_t nval,
              const std::vector<int32_t> *desc, int64_t ns, int M2) {
    if ((int64_t)ptr.size() != ns + 1 || ptr[0] != 0 || (size_t)ptr[ns] != col.size() || col.size() != nval)
        return fail(FSV_EINVAL, "internal: string Hamiltonian rows");
    for (int64_t I = 0; I < ns; ++I)
        if (ptr[I + 1] < ptr[I]) return fail(FSV_EINVAL, "internal: string Hamiltonian rows");
    for (int32_t c : col)
        if (c < 0 || c >= ns) return fail(FSV_EINVAL, "internal: string Hamiltonian column");
    if (desc) {
        if (desc->size() != nval) return fail(FSV_EINVAL, "internal: one-body descriptors");
        for (int32_t d : *desc)
            if ((d <= -2 && -2 - (int64_t)d >= ns) || (d >= 0 && (d & 0x3FFFFFFF) >= M2))
                return fail(FSV_EINVAL, "internal: one-body descriptor out of range");
    }
    return FSV_OK;
}

int bind_workspace(fsv_plan &P, void *base);

int build_device(fsv_plan &P) {
    int rc;
    init_kernels();
    HIPCHECK(hipStreamCreateWithFlags(&P.work, hipStreamNonBlocking));
    HIPCHECK(hipEventCreateWithFlags(&P.ev_in, hipEventDisableTiming));
    HIPCHECK(hipEventCreateWithFlags(&P.ev_out, hipEventDisableTiming));
    HIPCHECK(hipEventCreateWithFlags(&P.ev_cs, hipEventDisableTiming));
    const int M = P.M, G = max_grid();
    const size_t M2 = (size_t)M * M;
    P.pin_doubles = 2 * (size_t)P.K + (size_t)P.K + 1 + 4 * M2 + 8;
    HIPCHECK(hipHostMalloc((void **)&P.h_pin, sizeof(double) * P.pin_doubles, hipHostMallocDefault));
    HIPCHECK(hipHostMalloc((void **)&P.h_cs, sizeof(double) * (2 * (size_t)P.K + 2), hipHostMallocCoherent));

    // sector tables
    P.sa = strings_of(M, P.na);
    P.sb = strings_of(M, P.nb);
    P.nsa = (int64_t)P.sa.size();
    P.nsb = (int64_t)P.sb.size();
    P.dim = P.nsa * P.nsb;
    std::vector<int32_t> ra(1u << M, -1), rb(1u << M, -1);
    for (size_t i = 0; i < P.sa.size(); ++i) ra[P.sa[i]] = (int32_t)i;
    for (size_t i = 0; i < P.sb.size(); ++i) rb[P.sb[i]] = (int32_t)i;
    std::vector<uint64_t> Xa(P.nsa), Xb(P.nsb);
    std::vector<uint32_t> PPb(P.nsb);
    for (int64_t i = 0; i < P.nsa; ++i) {
        uint64_t x = 0;
        for (int p = 0; p < M; ++p)
            if (P.sa[i] >> p & 1u) x |= 1ull << qubit_of(P, 2 * p);
        Xa[i] = x;
    }
    for (int64_t i = 0; i < P.nsb; ++i) {
        uint64_t x = 0;
        uint32_t pp = 0;
        for (int p = 0; p < M; ++p)
            if (P.sb[i] >> p & 1u) x |= 1ull << qubit_of(P, 2 * p + 1);
        pp = beta_prefix_parity(M, P.ordering, P.sb[i]);
        Xb[i] = x;
        PPb[i] = pp;
    }
    P.PPb = PPb;
    P.ref_index = Xa[0] | Xb[0];  // strings are ascending: index 0 fills the lowest orbitals
    P.ref_phase = (__builtin_popcount(P.sa[0] & PPb[0]) & 1) ? -1.0 : 1.0;
    std::vector<uint32_t> excA, excB;
    build_exc(M, P.sa, ra, excA, P.nexcA);
    build_exc(M, P.sb, rb, excB, P.nexcB);
    std::vector<int32_t> boA, biA, boB, biB;
    build_bins(M, excA, P.nexcA, boA, biA);
    build_bins(M, excB, P.nexcB, boB, biB);
    std::vector<uint32_t> &plists = P.h_plists;
    plists.clear();
    P.pops.clear();
    for (int k = 0; k < P.K; ++k)
        P.pops.push_back(P.excitation ? build_pair_op_qeb(M, P.ordering, P.ops.data() + 4 * k, P.sa, ra, P.sb, rb, plists)
                                      : build_pair_op(M, P.ops.data() + 4 * k, P.sa, ra, P.sb, rb, plists));
    if ((rc = dalloc(P, &P.d_plists, plists.size()))) return rc;
    if ((rc = dalloc(P, &P.d_pops, (size_t)P.K))) return rc;
    if ((rc = dalloc(P, &P.d_ccount, (size_t)std::max(P.K, 1)))) return rc;
    if ((rc = upload(P, P.d_plists, plists.data(), plists.size()))) return rc;
    if ((rc = upload(P, P.d_pops, P.pops.data(), P.pops.size()))) return rc;
    P.fuse_mode = P.dim <= packet_default_dim() ? 3 : 0;
    if (const char *e = std::getenv("FSV_FUSE")) {
        if (!std::strcmp(e, "tiles")) P.fuse_mode = 0;
        if (!std::strcmp(e, "packets")) P.fuse_mode = 3;
    }
    if (const char *e = std::getenv("FSV_NO_FUSE")) P.fuse_mode = e[0] ? 1 : P.fuse_mode;
    if (std::getenv("FSV_FORCE_FUSE")) P.fuse_mode = 2;
    if ((rc = rebuild_fused(P))) return rc;
    if ((rc = check_tables(P, excA, excB, boA, biA, boB, biB))) return rc;

    if ((rc = dalloc(P, &P.d_rot, P.K))) return rc;
    if ((rc = dalloc(P, &P.d_cs, 2 * (size_t)P.K))) return rc;
    if ((rc = dalloc(P, &P.d_gcount, (size_t)P.K))) return rc;
    if ((rc = dalloc(P, &P.d_ecount, 1))) return rc;
    if ((rc = dalloc(P, &P.d_out, (size_t)P.K + 1))) return rc;
    if ((rc = dalloc(P, &P.d_Xa, P.nsa))) return rc;
    if ((rc = dalloc(P, &P.d_Xb, P.nsb))) return rc;
    if ((rc = dalloc(P, &P.d_sa, P.nsa))) return rc;
    if ((rc = dalloc(P, &P.d_PPb, P.nsb))) return rc;
    if ((rc = dalloc(P, &P.d_excA, excA.size()))) return rc;
    if ((rc = dalloc(P, &P.d_excB, excB.size()))) return rc;
    if ((rc = dalloc(P, &P.d_excBT, excB.size()))) return rc;
    if ((rc = dalloc(P, &P.d_g, M2 * M2))) return rc;
    if ((rc = dalloc(P, &P.d_binA_off, boA.size()))) return rc;
    if ((rc = dalloc(P, &P.d_binA_idx, biA.size()))) return rc;
    if ((rc = dalloc(P, &P.d_binB_off, boB.size()))) return rc;
    if ((rc = dalloc(P, &P.d_binB_idx, biB.size()))) return rc;

    if ((rc = upload(P, P.d_rot, P.rot.data(), P.rot.size()))) return rc;
    if ((rc = upload(P, P.d_Xa, Xa.data(), Xa.size()))) return rc;
    if ((rc = upload(P, P.d_Xb, Xb.data(), Xb.size()))) return rc;
    if ((rc = upload(P, P.d_sa, P.sa.data(), P.sa.size()))) return rc;
    if ((rc = upload(P, P.d_PPb, PPb.data(), PPb.size()))) return rc;
    if ((rc = upload(P, P.d_excA, excA.data(), excA.size()))) return rc;
    if ((rc = upload(P, P.d_excB, excB.data(), excB.size()))) return rc;
    {
        std::vector<uint32_t> excBT(excB.size());
        for (int64_t r = 0; r < P.nsb; ++r)
            for (int f = 0; f < P.nexcB; ++f) excBT[(size_t)f * P.nsb + r] = excB[(size_t)r * P.nexcB + f];
        if ((rc = upload(P, P.d_excBT, excBT.data(), excBT.size()))) return rc;
    }
    if ((rc = upload(P, P.d_g, P.g.data(), P.g.size()))) return rc;
    if ((rc = upload(P, P.d_binA_off, boA.data(), boA.size()))) return rc;
    if ((rc = upload(P, P.d_binA_idx, biA.data(), biA.size()))) return rc;
    if ((rc = upload(P, P.d_binB_off, boB.data(), boB.size()))) return rc;
    if ((rc = upload(P, P.d_binB_idx, biB.data(), biB.size()))) return rc;
    const int ec = (int)combine_grid(P.dim);
    if ((rc = upload(P, P.d_ecount, &ec, 1))) return rc;
    if ((rc = upload_counts(P))) return rc;

    // string Hamiltonians: structure and values
    std::vector<double> ht(P.h);
    build_string_h(M, P.sa, ra, ht.data(), P.g.data(), P.ha_ptr, P.ha_col, P.ha_val);
    build_string_h(M, P.sb, rb, ht.data(), P.g.data(), P.hb_ptr, P.hb_col, P.hb_val);
    if ((rc = check_csr(P.ha_ptr, P.ha_col, P.ha_val.size(), nullptr, P.nsa, (int)M2)) ||
        (rc = check_csr(P.hb_ptr, P.hb_col, P.hb_val.size(), nullptr, P.nsb, (int)M2)))
        return rc;
    if ((rc = dalloc(P, &P.d_ha_ptr, P.ha_ptr.size()))) return rc;
    if ((rc = dalloc(P, &P.d_ha_col, P.ha_col.size()))) return rc;
    if ((rc = dalloc(P, &P.d_ha_val, P.ha_val.size()))) return rc;
    if ((rc = dalloc(P, &P.d_hb_ptr, P.hb_ptr.size()))) return rc;
    if ((rc = dalloc(P, &P.d_hb_col, P.hb_col.size()))) return rc;
    if ((rc = dalloc(P, &P.d_hb_val, P.hb_val.size()))) return rc;
    if ((rc = upload(P, P.d_ha_ptr, P.ha_ptr.data(), P.ha_ptr.size()))) return rc;
    if ((rc = upload(P, P.d_ha_col, P.ha_col.data(), P.ha_col.size()))) return rc;
    if ((rc = upload(P, P.d_ha_val, P.ha_val.data(), P.ha_val.size()))) return rc;
    if ((rc = upload(P, P.d_hb_ptr, P.hb_ptr.data(), P.hb_ptr.size()))) return rc;
    if ((rc = upload(P, P.d_hb_col, P.hb_col.data(), P.hb_col.size()))) return rc;
    if ((rc = upload(P, P.d_hb_val, P.hb_val.data(), P.hb_val.size()))) return rc;
    {
        std::vector<double> zero((size_t)M * M, 0.0), v2;
        std::vector<int64_t> ptr2;
        std::vector<int32_t> col2, desc;
        auto part = [&](const std::vector<uint32_t> &str, const std::vector<int32_t> &rk, size_t nent,
                        double **d_v2, int32_t **d_desc, uint32_t **d_str) -> int {
            int r;
            build_string_h(M, str, rk, zero.data(), P.g.data(), ptr2, col2, v2);
            build_string_h_onebody(M, str, rk, desc);
            if (v2.size() != nent || desc.size() != nent)
                return fail(FSV_EINVAL, "internal: string Hamiltonian parts disagree");
            if ((r = check_csr(ptr2, col2, v2.size(), &desc, (int64_t)str.size(), (int)M2))) return r;
            if ((r = dalloc(P, d_v2, nent)) || (r = dalloc(P, d_desc, nent)) || (r = dalloc(P, d_str, str.size())))
                return r;
            if ((r = upload(P, *d_v2, v2.data(), nent)) || (r = upload(P, *d_desc, desc.data(), nent)) ||
                (r = upload(P, *d_str, str.data(), str.size())))
                return r;
            return FSV_OK;
        };
        if ((rc = part(P.sa, ra, P.ha_val.size(), &P.d_ha_v2, &P.d_ha_desc, &P.d_str_a)) ||
            (rc = part(P.sb, rb, P.hb_val.size(), &P.d_hb_v2, &P.d_hb_desc, &P.d_str_b)) ||
            (rc = dalloc(P, &P.d_htilde, (size_t)M * M)))
            return rc;
    }
    int R = 0;
    std::vector<double> Lt;
    choose_sigma(P, R, Lt);
    double *d_Lt = nullptr, *d_lda = nullptr, *d_ldb = nullptr;
    if (R > 0) {
        const int rp = lr_pad(R);
        const std::vector<double> da = diag_factor_sums(M, P.sa, Lt, rp), db = diag_factor_sums(M, P.sb, Lt, rp);
        if ((rc = dalloc(P, &d_Lt, Lt.size()))) return rc;
        if ((rc = upload(P, d_Lt, Lt.data(), Lt.size()))) return rc;
        if ((rc = dalloc(P, &d_lda, da.size())) || (rc = upload(P, d_lda, da.data(), da.size()))) return rc;
        if ((rc = dalloc(P, &d_ldb, db.size())) || (rc = upload(P, d_ldb, db.data(), db.size()))) return rc;
    }
    P.lr_R = R;
    {  // workspace layout (256-byte aligned parts)
        const size_t parts[9] = {16 * (size_t)P.dim, 16 * (size_t)P.dim, 16 * (size_t)P.dim, 16 * (size_t)P.dim,
                                 16 * (size_t)std::max<int64_t>(std::max(P.nsa * P.nexcA, P.nsb * P.nexcB), 1),
                                 16 * 2 * M2, R > 0 ? 16 * (size_t)lr_pad(R) * P.dim : 0,
                                 8 * (size_t)std::max(P.K, 1) * G, 8 * 1024};
        size_t at = 0;
        for (int i = 0; i < 9; ++i) {
            P.ws_off[i] = at;
            at += (parts[i] + 255) & ~(size_t)255;
        }
        P.ws_off[9] = at;
        P.ws_bytes = at;
    }
    if (want_dense_same_spin(P)) {
        if (rocblas_create_handle(&P.blas) != rocblas_status_success) {
            P.blas = nullptr;
            return fail(FSV_EDEVICE, "rocblas_create_handle failed");
        }
        if (rocblas_set_atomics_mode(P.blas, rocblas_atomics_not_allowed) != rocblas_status_success)
            return fail(FSV_EDEVICE, "rocblas_set_atomics_mode failed");
        if ((rc = dalloc(P, &P.d_ha_dense, (size_t)P.nsa * P.nsa))) return rc;
        if ((rc = dalloc(P, &P.d_hb_dense, (size_t)P.nsb * P.nsb))) return rc;
        if ((rc = dalloc(P, &P.d_hb_dense_t, (size_t)P.nsb * P.nsb))) return rc;
        if ((rc = refresh_dense_same_spin(P))) return rc;
    }
    P.tabs = SectorTabs{P.nsa, P.nsb, M, P.nexcA, P.nexcB, P.d_ha_ptr, P.d_hb_ptr, P.d_ha_col,
                        P.d_hb_col, P.d_ha_val, P.d_hb_val, P.d_excA, P.d_excB, P.d_excBT, P.d_g, P.ecore,
                        R, d_Lt, nullptr, P.d_ha_dense, P.d_hb_dense, (void *)P.blas, P.d_hb_dense_t,
                        d_lda, d_ldb, P.na, P.nb};
    {  // the scratch parts of energy_grad_noalloc (sector engine, real states)
        const bool f32 = P.svt == V_F32;
        const size_t parts[7] = {16 * (size_t)P.dim,                           // C: (psi, lam) pairs; FP32: widened psi
                                 f32 ? 8 * (size_t)P.dim : 0,                  // S: FP32 only, H psi in FP64
                                 8 * (size_t)P.dim, 8 * (size_t)P.dim,         // CT, ST: real transposes
                                 lr_uses_intermediate(P.tabs, false) ? 8 * (size_t)lr_pad(R) * P.dim : 0,
                                 8 * (size_t)std::max(P.K, 1) * G, 8 * 1024};
        size_t at = 0;
        for (int i = 0; i < 7; ++i) {
            P.na_off[i] = at;
            at += (parts[i] + 255) & ~(size_t)255;
        }
        P.na_off[7] = at;
    }
    if (P.blas) {
        // one eager product per amplitude type on a temporary workspace, outside
        // any capture, so that the GEMM library has loaded its kernels and sized
        // its own workspace before any call of the plan (captured or not)
        void *tmp = nullptr;
        const hipError_t e = hipMalloc(&tmp, P.ws_bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(FSV_ENOMEM, "hipMalloc of %zu bytes failed: %s", P.ws_bytes, hipGetErrorString(e));
        }
        rc = bind_workspace(P, tmp);
        P.ws = nullptr;
        (void)hipFree(tmp);
        if (rc) return rc;
    }
    return FSV_OK;
}

// Point the workspace parts into the block at base (device, ws_bytes).
// Captured graphs name the old parts, so they are dropped.
int bind_workspace(fsv_plan &P, void *base) {
    char *b = (char *)base;
    P.ws = base;
    P.d_C = (double2 *)(b + P.ws_off[0]);
    P.d_S = (double2 *)(b + P.ws_off[1]);
    P.d_CT = (double2 *)(b + P.ws_off[2]);
    P.d_ST = (double2 *)(b + P.ws_off[3]);
    P.d_O = (double2 *)(b + P.ws_off[4]);
    P.d_gamma = (double2 *)(b + P.ws_off[5]);
    P.d_YT = P.lr_R > 0 ? (double2 *)(b + P.ws_off[6]) : nullptr;
    P.d_gpart = (double *)(b + P.ws_off[7]);
    P.d_epart = (double *)(b + P.ws_off[8]);
    P.tabs.YT = P.d_YT;
    drop_graphs(P);
    if (P.blas && !P.ws_warm) {
        // one eager product per amplitude type, outside any graph capture, so
        // that the GEMM library has loaded its kernels and sized its own
        // workspace before the first capture (the work buffers hold no state)
        HIPCHECK(launch_fill_zero(P.d_C, (size_t)P.dim * sizeof(double2), P.work));
        HIPCHECK(launch_sector_sigma(false, P.tabs, P.d_C, P.d_S, P.d_CT, P.d_ST, P.d_epart, P.work));
        HIPCHECK(launch_sector_sigma(true, P.tabs, P.d_C, P.d_S, P.d_CT, P.d_ST, P.d_epart, P.work));
        HIPCHECK(hipStreamSynchronize(P.work));
        P.ws_warm = true;
    }
    return FSV_OK;
}

void release_workspace(fsv_plan &P) {
    if (P.ws_owned && P.ws) (void)hipFree(P.ws);
    P.ws = nullptr;
    P.ws_owned = false;
}

// The workspace of a call: the caller's block, or the plan's own, allocated
// on the first call that needs one.
int need_workspace(fsv_plan &P) {
    if (P.ws) return FSV_OK;
    void *p = nullptr;
    const hipError_t e = hipMalloc(&p, P.ws_bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        return fail(FSV_ENOMEM, "hipMalloc of the %zu-byte plan workspace failed: %s", P.ws_bytes,
                    hipGetErrorString(e));
    }
    P.ws_owned = true;
    const int rc = bind_workspace(P, p);
    if (rc) release_workspace(P);
    return rc;
}

}  // namespace

fsv_plan::~fsv_plan() {
    for (fsv_pool *q : pools) q->plan = nullptr;
    drop_graphs(*this);
    release_workspace(*this);
    for (void *p : init_mem) (void)hipFree(p);
    if (blas) (void)rocblas_destroy_handle(blas);
    for (auto &b : bufs) (void)hipFree(b.p);
    if (h_pin) (void)hipHostFree(h_pin);
    if (h_cs) (void)hipHostFree(h_cs);
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (ev_cs) (void)hipEventDestroy(ev_cs);
    if (work) (void)hipStreamDestroy(work);
}

namespace {

// Sector engine: time whole energy + gradient evaluations (graph launches)
// for candidate LDS budgets of the fused runs, and keep the fastest.
int autotune_sector(fsv_plan &P, void *psi, void *lam, std::string &rep) {
    struct Cand { int mode; size_t fwd, rev; };
    std::vector<Cand> cands = {{1, 0, 0},          {0, 32768, 65536},   {0, 49152, 98304},
                               {0, 65536, 98304},  {0, 65536, 131072},  {0, 98304, 163840},
                               {0, 163840, 163840}};
    if (P.dim <= packet_default_dim()) cands.push_back({3, 0, 0});
    const Cand keep{P.fuse_mode, P.fuse_budget_fwd, P.fuse_budget_rev};
    std::vector<double> th(P.K, 0.1);
    int rc;
    if ((rc = stage_theta(P, th.data()))) return rc;
    hipEvent_t e0, e1;
    HIPCHECK(hipEventCreate(&e0));
    HIPCHECK(hipEventCreate(&e1));
    auto apply = [&](const Cand &c) {
        P.fuse_mode = c.mode;
        P.fuse_budget_fwd = c.fwd ? c.fwd : keep.fwd;
        P.fuse_budget_rev = c.rev ? c.rev : keep.rev;
        return rebuild_fused(P);
    };
    rep.clear();
    char line[200];
    float best = 1e30f;
    Cand bestc = keep;
    for (const Cand &c : cands) {
        if ((rc = apply(c))) break;
        float ms = 1e30f;
        for (int r = 0; r < 4 && !rc; ++r) {  // the first launch also captures the graph
            float t = 0.f;
            if (hipEventRecord(e0, P.work) != hipSuccess) rc = fail(FSV_EDEVICE, "event record failed");
            if (!rc) rc = launch_energy_grad(P, psi, lam);
            if (!rc && (hipEventRecord(e1, P.work) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                        hipEventElapsedTime(&t, e0, e1) != hipSuccess))
                rc = fail(FSV_EDEVICE, "event timing failed");
            if (r > 0) ms = std::min(ms, t);
        }
        if (rc) break;
        int fo = 0, ro = 0;
        const int fr = fused_runs(P.ffwd, &fo), rr = fused_runs(P.frev, &ro);
        if (c.mode == 1)
            snprintf(line, sizeof line, "one launch per operator: %.3f ms\n", ms);
        else if (c.mode == 3)
            snprintf(line, sizeof line, "component packets: %d runs (%d ops): %.3f ms\n", rr, ro, ms);
        else
            snprintf(line, sizeof line,
                     "fused runs, LDS %zu / %zu KiB: forward %d runs (%d ops), adjoint %d runs (%d ops): %.3f ms\n",
                     c.fwd / 1024, c.rev / 1024, fr, fo, rr, ro, ms);
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
    snprintf(line, sizeof line, "chosen: %s, LDS %zu / %zu KiB\n",
             bestc.mode == 1 ? "per operator" : (bestc.mode == 3 ? "component packets" : "fused runs"),
             P.fuse_budget_fwd / 1024, P.fuse_budget_rev / 1024);
    rep += line;
    return FSV_OK;
}

}  // namespace

// ==================================================================== C ABI ==
extern "C" {

const char *fsv_last_error(void) { return g_err.c_str(); }

int fsv_plan_create(fsv_plan **out, const fsv_problem *p, void *hip_stream) {
    if (!out) return fail(FSV_EINVAL, "out is NULL");
    *out = nullptr;
    int rc = validate_problem(p);
    if (rc) return rc;
    fsv_plan *P = new (std::nothrow) fsv_plan();
    if (!P) return fail(FSV_ENOMEM, "plan allocation failed");
    P->n = p->n_qubits;
    P->M = p->n_qubits / 2;
    P->na = p->n_alpha;
    P->nb = p->n_beta;
    P->ordering = p->ordering;
    P->precision = p->precision;
    P->K = p->n_ops;
    P->ecore = p->e_core;
    P->amp_bytes = p->precision == 0 ? 16 : 8;
    P->svt = p->precision == 0 ? V_F64 : V_F32;
    P->wide = P->n > 31;
    const size_t M2 = (size_t)P->M * P->M;
    P->h.assign(p->h, p->h + M2);
    P->g.assign(p->g, p->g + M2 * M2);
    P->v.assign(M2, 0.0);
    P->ops.assign(p->ops, p->ops + 4 * (size_t)P->K);
    P->user = (hipStream_t)hip_stream;
    P->use_graph = std::getenv("FSV_NO_GRAPH") == nullptr;
    if (const char *e = std::getenv("FSV_ENGINE")) P->engine = std::strcmp(e, "dense") == 0 ? 1 : 0;
    P->excitation = p->excitation;
    for (int k = 0; k < P->K; ++k) {
        P->rot.push_back(compile_op(P->M, P->ordering, P->ops.data() + 4 * k, P->excitation));
        P->npairs.push_back(1ull << (P->n - P->rot.back().nt));
    }
    plan_segments(*P);
    rc = build_device(*P);
    if (rc) {
        delete P;
        return rc;
    }
    *out = P;
    clear_error();
    return FSV_OK;
}

int fsv_plan_destroy(fsv_plan *P) {
    if (!P) return FSV_OK;
    if (P->work) (void)hipStreamSynchronize(P->work);
    delete P;
    return FSV_OK;
}

size_t fsv_state_bytes(const fsv_plan *P) {
    if (!P) return 0;
    return ((size_t)1 << P->n) * (size_t)P->amp_bytes;
}

size_t fsv_plan_workspace_bytes(const fsv_plan *P) { return P ? P->ws_bytes : 0; }

size_t fsv_plan_device_bytes(const fsv_plan *P) {
    if (!P) return 0;
    size_t t = 0;
    for (const DevBuf &b : P->bufs) t += b.bytes;
    t += P->frev.bytes;                  // the forward schedule shares these or
    if (P->ffwd.mem != P->frev.mem) t += P->ffwd.bytes;  // holds its own
    t += 32 * (size_t)P->n_init;         // initial-state lists (4 x 8 bytes per determinant)
    if (P->ws_owned) t += P->ws_bytes;
    return t;
}

int fsv_plan_set_workspace(fsv_plan *P, void *ws_dev, size_t bytes) {
    if (!P) return fail(FSV_EINVAL, "plan is NULL");
    if (ws_dev && bytes < P->ws_bytes)
        return fail(FSV_EINVAL, "workspace of %zu bytes; the plan needs %zu", bytes, P->ws_bytes);
    if (ws_dev && ((uintptr_t)ws_dev & 255))
        return fail(FSV_EINVAL, "the workspace must be 256-byte aligned");
    if (ws_dev == P->ws) return FSV_OK;
    if (P->work) HIPCHECK(hipStreamSynchronize(P->work));
    release_workspace(*P);
    drop_graphs(*P);
    if (!ws_dev) return FSV_OK;  // the plan allocates its own on the next call
    const int rc = bind_workspace(*P, ws_dev);
    if (rc) P->ws = nullptr;
    return rc;
}

int fsv_plan_info(const fsv_plan *P, int64_t *nsa, int64_t *nsb, uint64_t *ref) {
    if (!P) return fail(FSV_EINVAL, "plan is NULL");
    if (nsa) *nsa = P->nsa;
    if (nsb) *nsb = P->nsb;
    if (ref) *ref = P->ref_index;
    return FSV_OK;
}

int fsv_plan_set_engine(fsv_plan *P, int engine) {
    if (!P) return fail(FSV_EINVAL, "plan is NULL");
    if (engine != 0 && engine != 1) return fail(FSV_EINVAL, "engine must be 0 (sector) or 1 (dense)");
    if (engine != P->engine) {
        if (P->work) HIPCHECK(hipStreamSynchronize(P->work));
        drop_graphs(*P);
        P->engine = engine;
    }
    return FSV_OK;
}

int fsv_plan_runs(const fsv_plan *P, int adjoint, int32_t *run_start, int32_t *fused_tiles) {
    if (!P) return fail(FSV_EINVAL, "plan is NULL");
    if (adjoint != 0 && adjoint != 1) return fail(FSV_EINVAL, "adjoint must be 0 or 1");
    const FusedSched &S = adjoint ? P->frev : P->ffwd;
    for (const FGroup &g : S.groups)
        for (int k = g.k0; k < g.k0 + g.nops; ++k) {
            if (run_start) run_start[k] = g.k0;
            if (fused_tiles)
                fused_tiles[k] = g.fused == 2 ? g.n_packets : (g.fused ? g.n_orbits * g.n_blocks : 0);
        }
    return (int)S.groups.size();
}


int fsv_time_runs(fsv_plan *P, int adjoint, void *psi, void *lam, float *ms) {
    if (!P || !psi || !ms || (adjoint && !lam)) return fail(FSV_EINVAL, "plan, psi, lam or ms is NULL");
    if (adjoint != 0 && adjoint != 1) return fail(FSV_EINVAL, "adjoint must be 0 or 1");
    if (P->engine != 0) return fail(FSV_ESTATE, "per-run timing is available on the sector engine only");
    int rc;
    if ((rc = fence_in(*P))) return rc;
    if ((rc = need_workspace(*P))) return rc;
    if ((rc = time_sweep_sector(*P, adjoint, psi, lam, ms))) return rc;
    if ((rc = fence_out(*P))) return rc;
    return (int)(adjoint ? P->frev : P->ffwd).groups.size();
}

int fsv_set_theta(fsv_plan *P, const double *theta) {
    if (!P) return fail(FSV_EINVAL, "plan is NULL");
    // the angles go to the plan's own buffer on its own stream, ahead of the
    // sweeps queued after this call; no caller data is read or written
    return upload_theta(*P, theta);
}

int fsv_forward_async(fsv_plan *P, void *psi) {
    if (!P || !psi) return fail(FSV_EINVAL, "plan or psi is NULL");
    int rc;
    if ((rc = fence_in(*P))) return rc;
    if ((rc = need_workspace(*P))) return rc;
    if ((rc = enq_forward(*P, psi))) return rc;
    return fence_out(*P);
}

int fsv_sigma_async(fsv_plan *P, const void *psi, void *lam) {
    if (!P || !psi || !lam) return fail(FSV_EINVAL, "plan, psi or lam is NULL");
    int rc;
    if ((rc = fence_in(*P))) return rc;
    if ((rc = need_workspace(*P))) return rc;
    if ((rc = enq_sigma(*P, psi, lam))) return rc;
    return fence_out(*P);
}

int fsv_reverse_async(fsv_plan *P, void *psi, void *lam) {
    if (!P || !psi || !lam) return fail(FSV_EINVAL, "plan, psi or lam is NULL");
    int rc;
    if ((rc = fence_in(*P))) return rc;
    if ((rc = need_workspace(*P))) return rc;
    if ((rc = enq_reverse(*P, psi, lam))) return rc;
    return fence_out(*P);
}

int fsv_finish(fsv_plan *P, double *E_out, double *grad_out) {
    if (!P) return fail(FSV_EINVAL, "plan is NULL");
    int rc;
    if ((rc = fence_in(*P))) return rc;
    if ((rc = download_out(*P, E_out, grad_out, true))) return rc;
    return FSV_OK;  // the host has waited for the plan's work
}

int ansatz_apply(fsv_plan *P, const double *theta, void *psi) {
    if (!P || !psi) return fail(FSV_EINVAL, "plan or psi is NULL");
    int rc;
    if ((rc = fence_in(*P, true))) return rc;
    if ((rc = need_workspace(*P))) return rc;
    if ((rc = upload_theta(*P, theta))) return rc;
    if ((rc = enq_ansatz_dense_out(*P, psi))) return rc;
    HIPCHECK(hipStreamSynchronize(P->work));
    return FSV_OK;  // the host has waited for this call's work
}

int energy(fsv_plan *P, const void *psi, double *E_out) {
    if (!P || !psi || !E_out) return fail(FSV_EINVAL, "plan, psi or E_out is NULL");
    int rc;
    if ((rc = fence_in(*P, true))) return rc;
    if ((rc = need_workspace(*P))) return rc;
    if ((rc = enq_sigma_dense(*P, psi, nullptr))) return rc;
    if ((rc = download_out(*P, E_out, nullptr, false))) return rc;
    return FSV_OK;  // the host has waited for this call's work
}

int energy_grad(fsv_plan *P, const double *theta, void *psi, void *lam, double *E_out,
                double *grad_out) {
    if (!P || !psi || !lam) return fail(FSV_EINVAL, "plan, psi or lam is NULL");
    if (psi == lam) return fail(FSV_EINVAL, "psi and lam must be distinct buffers");
    if (P->K > 0 && !grad_out) return fail(FSV_EINVAL, "grad_out is NULL");
    int rc;
    if ((rc = fence_in(*P, true))) return rc;
    if ((rc = need_workspace(*P))) return rc;
    if ((rc = stage_theta(*P, theta))) return rc;
    if ((rc = launch_energy_grad(*P, psi, lam))) return rc;
    if ((rc = download_out(*P, E_out, grad_out, true))) return rc;
    return FSV_OK;  // the host has waited for this call's work
}

int energy_grad_noalloc(fsv_plan *P, const double *theta, void *psi, void *lam, double *E_out,
                        double *grad_out) {
    if (!P || !psi || !lam) return fail(FSV_EINVAL, "plan, psi or lam is NULL");
    if (psi == lam) return fail(FSV_EINVAL, "psi and lam must be distinct buffers");
    if (P->K > 0 && !grad_out) return fail(FSV_EINVAL, "grad_out is NULL");
    if (P->engine != 0) return fail(FSV_ESTATE, "energy_grad_noalloc runs on the sector engine");
    if (P->na_off[7] > kScratchBytes)
        return fail(FSV_EINVAL, "this plan needs %zu bytes of scratch; energy_grad_noalloc has %zu", P->na_off[7],
                    kScratchBytes);
    void *base = nullptr;
    int rc;
    if ((rc = scratch_address(&base))) return rc;
    if ((rc = fence_in(*P, true))) return rc;
    if ((rc = upload_theta(*P, theta))) return rc;
    // the pass takes its parts from the scratch block: the plan's workspace
    // fields point there for the duration of the (eager) launches
    char *b = (char *)base;
    double2 *sv[5] = {P->d_C, P->d_S, P->d_CT, P->d_ST, P->d_YT};
    double *sg = P->d_gpart, *se = P->d_epart;
    void *syt = P->tabs.YT;
    P->d_C = (double2 *)(b + P->na_off[0]);
    P->d_S = (double2 *)(b + P->na_off[1]);
    P->d_CT = (double2 *)(b + P->na_off[2]);
    P->d_ST = (double2 *)(b + P->na_off[3]);
    P->d_YT = (double2 *)(b + P->na_off[4]);
    P->tabs.YT = P->d_YT;
    P->d_gpart = (double *)(b + P->na_off[5]);
    P->d_epart = (double *)(b + P->na_off[6]);
    rc = run_energy_grad_body(*P, psi, lam);
    P->d_C = sv[0];
    P->d_S = sv[1];
    P->d_CT = sv[2];
    P->d_ST = sv[3];
    P->d_YT = sv[4];
    P->tabs.YT = syt;
    P->d_gpart = sg;
    P->d_epart = se;
    if (rc) return rc;
    if ((rc = download_out(*P, E_out, grad_out, true))) return rc;
    return FSV_OK;  // the host has waited for this call's work
}

int energy_grad_fd(fsv_plan *P, const double *theta, double step, void *psi, double *E_out,
                   double *grad_out) {
    if (!P || !psi || !theta) return fail(FSV_EINVAL, "plan, theta or psi is NULL");
    if (!(step > 0.0) || !std::isfinite(step)) return fail(FSV_EINVAL, "step must be > 0");
    if (P->K > 0 && !grad_out) return fail(FSV_EINVAL, "grad_out is NULL");
    int rc;
    if ((rc = fence_in(*P, true))) return rc;
    if ((rc = need_workspace(*P))) return rc;
    std::vector<double> th(theta, theta + P->K);
    double e0 = 0.0;
    if ((rc = upload_theta(*P, th.data()))) return rc;
    if ((rc = launch_energy_only(*P, psi))) return rc;
    if ((rc = download_out(*P, &e0, nullptr, false))) return rc;
    for (int k = 0; k < P->K; ++k) {
        double ep = 0.0, em = 0.0;
        th[k] = theta[k] + step;
        if ((rc = upload_theta(*P, th.data()))) return rc;
        if ((rc = launch_energy_only(*P, psi))) return rc;
        if ((rc = download_out(*P, &ep, nullptr, false))) return rc;
        th[k] = theta[k] - step;
        if ((rc = upload_theta(*P, th.data()))) return rc;
        if ((rc = launch_energy_only(*P, psi))) return rc;
        if ((rc = download_out(*P, &em, nullptr, false))) return rc;
        th[k] = theta[k];
        grad_out[k] = (ep - em) / (2.0 * step);
    }
    if (E_out) *E_out = e0;
    return FSV_OK;  // the host has waited for this call's work
}

int rdm1(fsv_plan *P, const void *psi, double *gamma_out) {
    if (!P || !psi || !gamma_out) return fail(FSV_EINVAL, "plan, psi or gamma_out is NULL");
    int rc;
    if ((rc = fence_in(*P, true))) return rc;
    if ((rc = need_workspace(*P))) return rc;
    hipStream_t st = P->work;
    const int M2 = P->M * P->M;
    HIPCHECK(launch_gather(P->precision, psi, P->d_Xa, P->d_Xb, P->d_sa, P->d_PPb, P->nsa, P->nsb, P->d_C, st));
    if (P->nexcA > 0) {
        HIPCHECK(launch_rdm_overlap(P->d_C, P->nsa, P->nsb, P->d_excA, P->nexcA, P->d_O, st));
        HIPCHECK(launch_rdm_bin(P->d_O, P->d_binA_off, P->d_binA_idx, M2, P->d_gamma, st));
    } else {
        HIPCHECK(launch_fill_zero(P->d_gamma, sizeof(double2) * M2, st));
    }
    HIPCHECK(launch_ctranspose(true, P->d_C, P->d_CT, P->nsa, P->nsb, st));
    if (P->nexcB > 0) {
        HIPCHECK(launch_rdm_overlap(P->d_CT, P->nsb, P->nsa, P->d_excB, P->nexcB, P->d_O, st));
        HIPCHECK(launch_rdm_bin(P->d_O, P->d_binB_off, P->d_binB_idx, M2, P->d_gamma + M2, st));
    } else {
        HIPCHECK(launch_fill_zero(P->d_gamma + M2, sizeof(double2) * M2, st));
    }
    double *h = P->h_pin + 3 * (size_t)P->K + 1;
    HIPCHECK(hipMemcpyAsync(h, P->d_gamma, sizeof(double2) * 2 * M2, hipMemcpyDeviceToHost, st));
    HIPCHECK(hipStreamSynchronize(st));
    std::memcpy(gamma_out, h, sizeof(double2) * 2 * M2);
    return FSV_OK;  // the host has waited for this call's work
}

int set_onebody_potential(fsv_plan *P, const double *v) {
    if (!P) return fail(FSV_EINVAL, "plan is NULL");
    const int M = P->M;
    if (v) {
        if (!finite_all(v, (size_t)M * M)) return fail(FSV_ENONFINITE, "non-finite v");
        double scale = 1.0;
        for (int i = 0; i < M * M; ++i) scale = std::max(scale, std::fabs(v[i]));
        for (int a = 0; a < M; ++a)
            for (int b = 0; b < M; ++b)
                if (std::fabs(v[a * M + b] - v[b * M + a]) > 1e-12 * scale)
                    return fail(FSV_EINVAL, "v is not symmetric at (%d,%d)", a, b);
        P->v.assign(v, v + (size_t)M * M);
    } else {
        P->v.assign((size_t)M * M, 0.0);
    }
    int rc;
    if ((rc = fence_in(*P))) return rc;
    if ((rc = upload_hamiltonian_values(*P))) return rc;
    return fence_out(*P);
}

int fsv_autotune(fsv_plan *P, void *psi, void *lam, const char **report) {
    static thread_local std::string rep;
    if (!P || !psi || !lam) return fail(FSV_EINVAL, "plan, psi or lam is NULL");
    if (psi == lam) return fail(FSV_EINVAL, "psi and lam must be distinct buffers");
    int rc;
    if ((rc = fence_in(*P))) return rc;
    if ((rc = need_workspace(*P))) return rc;
    if (P->engine == 0) {
        if ((rc = autotune_sector(*P, psi, lam, rep))) return rc;
        if (report) *report = rep.c_str();
        return fence_out(*P);
    }
    const char *cache = std::getenv("FSV_TUNE_CACHE");
    char key[128];
    snprintf(key, sizeof key, "n%d_p%d_o%d_K%d", P->n, P->precision, P->ordering, P->K);
    if (cache) {
        FILE *f = fopen(cache, "r");
        if (f) {
            char k2[128];
            int b1, p1, b2, p2;
            while (fscanf(f, "%127s %d %d %d %d", k2, &b1, &p1, &b2, &p2) == 5) {
                if (std::strcmp(k2, key) == 0) {
                    P->shape_rot = {b1, p1};
                    P->shape_adj = {b2, p2};
                    fclose(f);
                    drop_graphs(*P);
                    if ((rc = upload_counts(*P))) return rc;
                    rep = std::string("cached ") + key;
                    if (report) *report = rep.c_str();
                    return fence_out(*P);
                }
            }
            fclose(f);
        }
    }
    std::vector<double> th(P->K, 0.1);
    if ((rc = upload_theta(*P, th.data()))) return rc;
    hipEvent_t e0, e1;
    HIPCHECK(hipEventCreate(&e0));
    HIPCHECK(hipEventCreate(&e1));
    const Shape cands[] = {{256, 1}, {256, 2}, {256, 4}, {256, 8}, {512, 2}, {512, 4}, {128, 4}, {1024, 2}};
    float best_f = 1e30f, best_r = 1e30f;
    Shape bf = P->shape_rot, br = P->shape_adj;
    char line[160];
    rep.clear();
    const int nk = std::min(P->K, 64);
    for (const Shape &sh : cands) {
        // forward rotations
        for (int rep_i = 0; rep_i < 2; ++rep_i) {
            HIPCHECK(hipEventRecord(e0, P->work));
            for (int k = 0; k < nk; ++k)
                HIPCHECK(launch_rot(P->precision, P->wide, psi, P->rot[k], P->d_cs, k, P->npairs[k], sh, P->work));
            HIPCHECK(hipEventRecord(e1, P->work));
            HIPCHECK(hipEventSynchronize(e1));
        }
        float tf = 0.f;
        HIPCHECK(hipEventElapsedTime(&tf, e0, e1));
        float tr = 0.f;
        for (int rep_i = 0; rep_i < 2; ++rep_i) {
            HIPCHECK(hipEventRecord(e0, P->work));
            for (int k = 0; k < nk; ++k)
                HIPCHECK(launch_adj(P->precision, P->wide, psi, lam, P->rot[k], P->d_cs, k, P->npairs[k], sh,
                                    P->d_gpart + (size_t)k * max_grid(), P->work));
            HIPCHECK(hipEventRecord(e1, P->work));
            HIPCHECK(hipEventSynchronize(e1));
        }
        HIPCHECK(hipEventElapsedTime(&tr, e0, e1));
        snprintf(line, sizeof line, "block %d ppt %d: rot %.3f ms adj %.3f ms (%d ops)\n", sh.block,
                 sh.ppt, tf, tr, nk);
        rep += line;
        if (tf < best_f) { best_f = tf; bf = sh; }
        if (tr < best_r) { best_r = tr; br = sh; }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    P->shape_rot = bf;
    P->shape_adj = br;
    drop_graphs(*P);
    if ((rc = upload_counts(*P))) return rc;
    snprintf(line, sizeof line, "chosen rot (%d,%d) adj (%d,%d)\n", bf.block, bf.ppt, br.block, br.ppt);
    rep += line;
    if (cache) {
        FILE *f = fopen(cache, "a");
        if (f) {
            fprintf(f, "%s %d %d %d %d\n", key, bf.block, bf.ppt, br.block, br.ppt);
            fclose(f);
        }
    }
    if (report) *report = rep.c_str();
    return fence_out(*P);
}

// ------------------------------------------------- initial state, properties ----
int fsv_set_initial_state(fsv_plan *P, int32_t n_det, const uint64_t *dets, const double *coef) {
    if (!P) return fail(FSV_EINVAL, "plan is NULL");
    if (n_det < 0 || (n_det > 0 && (!dets || !coef))) return fail(FSV_EINVAL, "bad n_det / dets / coef");
    if (n_det > 0 && (int64_t)n_det > P->dim) return fail(FSV_EINVAL, "more determinants than the sector holds");
    if (!finite_all(coef, (size_t)n_det)) return fail(FSV_ENONFINITE, "non-finite coefficient");
    const int M = P->M;
    std::vector<int32_t> ra((size_t)1 << M, -1), rb((size_t)1 << M, -1);
    for (size_t i = 0; i < P->sa.size(); ++i) ra[P->sa[i]] = (int32_t)i;
    for (size_t i = 0; i < P->sb.size(); ++i) rb[P->sb[i]] = (int32_t)i;
    std::vector<int64_t> sidx(n_det), didx(n_det);
    std::vector<double> sval(n_det), dval(n_det);
    for (int d = 0; d < n_det; ++d) {
        const uint64_t x = dets[d];
        if (P->n < 64 && (x >> P->n) != 0) return fail(FSV_EINVAL, "determinant %d has bits above qubit %d", d, P->n - 1);
        uint32_t a = 0, b = 0;
        for (int p = 0; p < M; ++p) {
            a |= (uint32_t)((x >> qubit_of(*P, 2 * p)) & 1u) << p;
            b |= (uint32_t)((x >> qubit_of(*P, 2 * p + 1)) & 1u) << p;
        }
        if (ra[a] < 0 || rb[b] < 0)
            return fail(FSV_EINVAL, "determinant %d lies outside the (%d, %d) sector", d, P->na, P->nb);
        sidx[d] = (int64_t)ra[a] * P->nsb + rb[b];
        // the alpha-first sector amplitude is the qubit-basis amplitude times
        // (-1)^popcount(alpha string & beta prefix parity)
        sval[d] = (__builtin_popcount(a & P->PPb[rb[b]]) & 1) ? -coef[d] : coef[d];
        didx[d] = (int64_t)x;
        dval[d] = coef[d];
    }
    {
        std::vector<int64_t> srt(sidx);
        std::sort(srt.begin(), srt.end());
        for (size_t i = 1; i < srt.size(); ++i)
            if (srt[i] == srt[i - 1]) return fail(FSV_EINVAL, "a determinant is listed twice");
    }
    if (P->work) HIPCHECK(hipStreamSynchronize(P->work));
    drop_graphs(*P);  // captured launches point at the old list
    for (void *q : P->init_mem) (void)hipFree(q);
    P->init_mem.clear();
    P->n_init = 0;
    P->d_init_sidx = P->d_init_didx = nullptr;
    P->d_init_sval = P->d_init_dval = nullptr;
    if (n_det == 0) {
        clear_error();
        return FSV_OK;
    }
    void *bufs[4] = {nullptr, nullptr, nullptr, nullptr};
    const size_t bytes = 8 * (size_t)n_det;
    for (int i = 0; i < 4; ++i) {
        if (hipMalloc(&bufs[i], bytes) != hipSuccess) {
            (void)hipGetLastError();
            for (int j = 0; j < i; ++j) (void)hipFree(bufs[j]);
            return fail(FSV_ENOMEM, "hipMalloc of the initial state list failed");
        }
    }
    P->init_mem.assign(bufs, bufs + 4);
    P->d_init_sidx = (int64_t *)bufs[0];
    P->d_init_sval = (double *)bufs[1];
    P->d_init_didx = (int64_t *)bufs[2];
    P->d_init_dval = (double *)bufs[3];
    HIPCHECK(hipMemcpy(P->d_init_sidx, sidx.data(), bytes, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(P->d_init_sval, sval.data(), bytes, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(P->d_init_didx, didx.data(), bytes, hipMemcpyHostToDevice));
    HIPCHECK(hipMemcpy(P->d_init_dval, dval.data(), bytes, hipMemcpyHostToDevice));
    P->n_init = n_det;
    clear_error();
    return FSV_OK;
}

int onebody_expectation(fsv_plan *P, const void *psi, const double *d, double *out) {
    if (!P || !psi || !d || !out) return fail(FSV_EINVAL, "plan, psi, d or out is NULL");
    const int M = P->M;
    if (!finite_all(d, (size_t)M * M)) return fail(FSV_ENONFINITE, "non-finite d");
    std::vector<double> gam(4 * (size_t)M * M);
    int rc = rdm1(P, psi, gam.data());
    if (rc) return rc;
    double re = 0.0, im = 0.0;
    for (int s = 0; s < 2; ++s)
        for (int pq = 0; pq < M * M; ++pq) {
            re += d[pq] * gam[2 * ((size_t)s * M * M + pq)];
            im += d[pq] * gam[2 * ((size_t)s * M * M + pq) + 1];
        }
    out[0] = re;
    out[1] = im;
    return FSV_OK;
}

// ------------------------------------------------------------ pools ----
int fsv_pool_create(fsv_pool **out, fsv_plan *P, const int32_t *ops, int32_t n_ops, int32_t excitation) {
    if (!out) return fail(FSV_EINVAL, "out is NULL");
    *out = nullptr;
    if (!P) return fail(FSV_EINVAL, "plan is NULL");
    if (n_ops < 1 || n_ops > 65535) return fail(FSV_EINVAL, "a pool holds 1 .. 65535 operators");
    if (excitation != 0 && excitation != 1) return fail(FSV_EINVAL, "excitation must be 0 or 1");
    int rc = validate_ops(P->n, n_ops, ops);
    if (rc) return rc;
    if (P->engine != 0) return fail(FSV_ESTATE, "pool screening runs on the sector engine");
    fsv_pool *Q = new (std::nothrow) fsv_pool();
    if (!Q) return fail(FSV_ENOMEM, "pool allocation failed");
    Q->plan = P;
    Q->n = n_ops;
    std::vector<int32_t> ra((size_t)1 << P->M, -1), rb((size_t)1 << P->M, -1);
    for (size_t i = 0; i < P->sa.size(); ++i) ra[P->sa[i]] = (int32_t)i;
    for (size_t i = 0; i < P->sb.size(); ++i) rb[P->sb[i]] = (int32_t)i;
    std::vector<PairOp> pops;
    std::vector<uint32_t> lists;
    double maxpairs = 1.0;
    for (int t = 0; t < n_ops; ++t) {
        const int32_t *o = ops + 4 * t;
        const PairOp po = excitation ? build_pair_op_qeb(P->M, P->ordering, o, P->sa, ra, P->sb, rb, lists)
                                     : build_pair_op(P->M, o, P->sa, ra, P->sb, rb, lists);
        maxpairs = std::max(maxpairs, (double)(po.nA >= 0 ? po.nA : P->nsa) * (double)(po.nB >= 0 ? po.nB : P->nsb));
        pops.push_back(po);
    }
    for (int t = 0; t < n_ops; ++t)  // pair-list bounds, as for the plan's own operators
        for (int side = 0; side < 2; ++side) {
            const int32_t n = side ? pops[t].nB : pops[t].nA;
            const int64_t off = side ? pops[t].offB : pops[t].offA, ns = side ? P->nsb : P->nsa;
            bool good = n >= -1 && (n < 0 || off + n <= (int64_t)lists.size());
            for (int32_t u = 0; good && u < n; ++u)
                good = (int64_t)(lists[off + u] & 0x7FFFu) < ns && (int64_t)((lists[off + u] >> 15) & 0x7FFFu) < ns;
            if (!good) {
                delete Q;
                return fail(FSV_EINVAL, "internal: pair list of pool operator %d out of range", t);
            }
        }
    // workgroups per operator: ~16 pairs per thread for the largest, at most 64
    Q->gx = (int)std::min(64.0, std::max(1.0, std::ceil(maxpairs / (256.0 * 16.0))));
    auto dal = [&](void **p, size_t bytes) -> int {
        if (hipMalloc(p, std::max<size_t>(bytes, 4)) != hipSuccess) {
            (void)hipGetLastError();
            return fail(FSV_ENOMEM, "hipMalloc of %zu bytes for the pool failed", bytes);
        }
        Q->mem.push_back(*p);
        return FSV_OK;
    };
    std::vector<int> counts(n_ops, Q->gx);
    if ((rc = dal((void **)&Q->d_ops, sizeof(PairOp) * pops.size())) ||
        (rc = dal((void **)&Q->d_lists, 4 * lists.size())) ||
        (rc = dal((void **)&Q->d_part, sizeof(double) * (size_t)n_ops * Q->gx)) ||
        (rc = dal((void **)&Q->d_out, sizeof(double) * (size_t)n_ops)) ||
        (rc = dal((void **)&Q->d_counts, sizeof(int) * (size_t)n_ops))) {
        delete Q;
        return rc;
    }
    if (hipMemcpy(Q->d_ops, pops.data(), sizeof(PairOp) * pops.size(), hipMemcpyHostToDevice) != hipSuccess ||
        (!lists.empty() && hipMemcpy(Q->d_lists, lists.data(), 4 * lists.size(), hipMemcpyHostToDevice) != hipSuccess) ||
        hipMemcpy(Q->d_counts, counts.data(), sizeof(int) * counts.size(), hipMemcpyHostToDevice) != hipSuccess ||
        hipHostMalloc((void **)&Q->h_pin, sizeof(double) * ((size_t)n_ops + 1), hipHostMallocDefault) != hipSuccess) {
        (void)hipGetLastError();
        delete Q;
        return fail(FSV_EDEVICE, "pool upload failed");
    }
    P->pools.push_back(Q);
    *out = Q;
    clear_error();
    return FSV_OK;
}

int fsv_pool_destroy(fsv_pool *Q) {
    if (!Q) return FSV_OK;
    if (fsv_plan *P = Q->plan) {
        if (P->work) (void)hipStreamSynchronize(P->work);
        P->pools.erase(std::remove(P->pools.begin(), P->pools.end(), Q), P->pools.end());
    }
    delete Q;
    return FSV_OK;
}

int fsv_pool_gradients(fsv_pool *Q, const double *theta, void *psi, void *lam, double *E_out, double *grad_out) {
    if (!Q || !psi || !lam || !grad_out) return fail(FSV_EINVAL, "pool, psi, lam or grad_out is NULL");
    if (psi == lam) return fail(FSV_EINVAL, "psi and lam must be distinct buffers");
    if (!Q->plan) return fail(FSV_ESTATE, "the plan of this pool has been destroyed");
    fsv_plan &P = *Q->plan;
    if (P.engine != 0) return fail(FSV_ESTATE, "pool screening runs on the sector engine");
    int rc;
    if ((rc = fence_in(P, true))) return rc;
    if ((rc = need_workspace(P))) return rc;
    if ((rc = upload_theta(P, theta))) return rc;
    auto body = [&]() -> int {
        int r;
        if ((r = enq_forward(P, psi))) return r;
        if ((r = enq_sigma(P, psi, lam))) return r;
        HIPCHECK(launch_pool(P.svt, psi, lam, Q->d_ops, Q->d_lists, Q->n, Q->gx, P.nsa, P.nsb, Q->d_part, P.work));
        HIPCHECK(launch_reduce_rows(Q->d_part, Q->d_counts, Q->gx, Q->n, 2.0, Q->d_out, P.work));
        return FSV_OK;
    };
    if (!P.use_graph) {
        if ((rc = body())) return rc;
    } else {
        if (!Q->graph || Q->g_psi != psi || Q->g_lam != lam || Q->gen != P.gen) {
            if (Q->graph) (void)hipGraphExecDestroy(Q->graph);
            Q->graph = nullptr;
            if ((rc = capture(P, body, &Q->graph))) {
                Q->graph = nullptr;
                return rc;
            }
            Q->g_psi = psi;
            Q->g_lam = lam;
            Q->gen = P.gen;
        }
        HIPCHECK(hipGraphLaunch(Q->graph, P.work));
    }
    HIPCHECK(hipMemcpyAsync(Q->h_pin, P.d_out, sizeof(double), hipMemcpyDeviceToHost, P.work));
    HIPCHECK(hipMemcpyAsync(Q->h_pin + 1, Q->d_out, sizeof(double) * Q->n, hipMemcpyDeviceToHost, P.work));
    HIPCHECK(hipStreamSynchronize(P.work));
    if (E_out) *E_out = Q->h_pin[0];
    std::memcpy(grad_out, Q->h_pin + 1, sizeof(double) * Q->n);
    return FSV_OK;  // the host has waited for this call's work
}

// Batches are built in fsv_batch.hip.

}  // extern "C"
