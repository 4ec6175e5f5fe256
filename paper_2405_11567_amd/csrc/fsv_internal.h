// Internal declarations shared by the kernel file and the host library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <memory>
#include <vector>

#include "../../include/fsv.h"

namespace fsv {

// One excitation rotation compiled for the dense kernels.  The active source
// strings are base | src and their partners base | dst, where base has zeros
// at the nt sorted target qubits q[]; the JW sign of tau on the source is
// sign0 * (-1)^popcount(base & par).
struct RotOp {
    uint64_t src, dst, par;
    uint32_t q[4];
    int32_t nt;
    int32_t sign0;
};

// One excitation on the sector-compressed state C[Ia][Ib] (alpha-string-first
// product basis = blocked JW ordering restricted to the sector).  Its active
// pairs are the product of an alpha pair list and a beta pair list; a list
// length of -1 means "every string maps to itself with sign +1".  List entries
// pack the source string (bits 0..14), the partner (15..29) and a negative-sign
// flag (bit 31); the pair sign is sign0 times both flags.
struct PairOp {
    int32_t nA, nB;
    int64_t offA, offB;
    int32_t sign0, pad;
};

__host__ __device__ inline uint32_t pack_pair(uint32_t s, uint32_t d, int neg) {
    return s | (d << 15) | (neg ? 0x80000000u : 0u);
}

// Launch shape of the pair kernels.
struct Shape {
    int block;   // threads per workgroup
    int ppt;     // pairs per thread per loop trip (1, 2, 4, 8)
};

// Packed string excitation: bits 0..15 source string J, 16..24 p*M+q,
// bit 31 set for a negative sign.
__host__ __device__ inline uint32_t pack_exc(uint32_t J, uint32_t pq, int neg) {
    return J | (pq << 16) | (neg ? 0x80000000u : 0u);
}

// ---- host helpers shared by plans and batches (fsv_host.hip) ----
int fail(int code, const char *fmt, ...);
void clear_error();
// True when every operation queued on st has completed.  A query that fails
// for any other reason counts as pending, so that the caller fences.
inline bool stream_idle(hipStream_t st) {
    const hipError_t q = hipStreamQuery(st);
    if (q == hipSuccess) return true;
    (void)hipGetLastError();
    return false;
}
int validate_problem(const fsv_problem *p);
int validate_ops(int n_qubits, int n_ops, const int32_t *ops);
// excitation 1: a qubit excitation (no JW string: sign +1 on every pair)
RotOp compile_op(int M, int ordering, const int32_t *op, int excitation = 0);
std::vector<uint32_t> strings_of(int M, int N);  // popcount-N masks, ascending
// Prefix-parity mask of a beta string b (M spatial orbitals) for a qubit
// ordering (0: qubit 2p + s, 1: qubit p + s M): bit q is set when an odd
// number of b's occupied beta orbitals sit on qubits below alpha orbital q's
// qubit.  (-1)^popcount(a & mask) is the sign between the qubit-basis
// amplitude of determinant (a, b) and its alpha-first sector amplitude.
uint32_t beta_prefix_parity(int M, int ordering, uint32_t b);
void build_string_h(int M, const std::vector<uint32_t> &str, const std::vector<int32_t> &rank,
                    const double *ht, const double *g, std::vector<int64_t> &ptr,
                    std::vector<int32_t> &col, std::vector<double> &val);
// Per string (ascending rank): its excitations p -> q, q empty, then its
// diagonal entries p -> p (the last popcount entries), as packed words.
void build_exc(int M, const std::vector<uint32_t> &str, const std::vector<int32_t> &rank,
               std::vector<uint32_t> &exc, int &nexc);
// Per string: the factor rows Lt[pp][0..rp) of its occupied p summed (its
// diagonal excitations folded into one), nstr x rp.
std::vector<double> diag_factor_sums(int M, const std::vector<uint32_t> &str, const std::vector<double> &Lt, int rp);
// Pivoted Cholesky of a symmetric positive semidefinite n x n matrix:
// G ~ sum_k L_k L_k^T with R rows of L (length n); returns R, or -1 when G is
// not positive semidefinite within tol * max(diag).
int pivoted_cholesky(int n, const double *G, double tol, std::vector<double> &L);
// Pair lists of one operator for the sector-compressed state; appends to lists.
PairOp build_pair_op(int M, const int32_t *op, const std::vector<uint32_t> &sa,
                     const std::vector<int32_t> &ra, const std::vector<uint32_t> &sb,
                     const std::vector<int32_t> &rb, std::vector<uint32_t> &lists);
// The same for a qubit excitation in the given qubit ordering.
PairOp build_pair_op_qeb(int M, int ordering, const int32_t *op, const std::vector<uint32_t> &sa,
                         const std::vector<int32_t> &ra, const std::vector<uint32_t> &sb,
                         const std::vector<int32_t> &rb, std::vector<uint32_t> &lists);

// ---- launchers (fsv_kernels.hip) ----
// precision: 0 complex128, 1 complex64.  Each returns the hipError_t of the launch.
int max_grid();
void init_kernels();  // once per process, before any capture (sets kernel attributes)

hipError_t launch_fill_zero(void *ptr, size_t bytes, hipStream_t st);
hipError_t launch_set_amp(void *psi, int vtype, uint64_t x, double re, hipStream_t st);
hipError_t launch_copy_doubles(const double *src, double *dst, int n, hipStream_t st);
// psi[idx[i]] = (val[i], 0) for i < n; vtype selects the storage (VType).
hipError_t launch_set_list(void *psi, int vtype, const int64_t *idx, const double *val, int n, hipStream_t st);

// Grid used for op with npairs pairs under shape sh (fixed per op: reductions
// depend on it).
unsigned rot_grid(uint64_t npairs, Shape sh);

hipError_t launch_rot(int precision, bool wide, void *psi, const RotOp &op, const double *cs,
                      int k, uint64_t npairs, Shape sh, hipStream_t st);
hipError_t launch_adj(int precision, bool wide, void *psi, void *lam, const RotOp &op,
                      const double *cs, int k, uint64_t npairs, Shape sh, double *partial,
                      hipStream_t st);
// LDS-staged fused run: ops [k0, k1) whose targets all lie below tile_bits are
// applied block by block in one pass over psi (+theta in order).
hipError_t launch_rot_fused(int precision, void *psi, const RotOp *ops_dev, const double *cs,
                            int k0, int k1, int tile_bits, uint64_t n_amps, hipStream_t st);
// Its adjoint: one pass over psi and lam undoes ops k1-1 .. k0 and writes each
// operator's gradient partials to partial[k * pstride + b], b < fused_grid().
// At most max_fused_run() operators.
hipError_t launch_adj_fused(int precision, void *psi, void *lam, const RotOp *ops_dev, const double *cs,
                            int k0, int k1, int tile_bits, uint64_t n_amps, double *partial, int pstride,
                            hipStream_t st);
unsigned fused_grid(uint64_t n_amps, int tile_bits);
int max_fused_run();

// out[0] = the energy partials' sum, out[1 + k] = 2 x operator k's gradient
// partials' sum (rows as in launch_reduce_rows), one launch.
hipError_t launch_reduce_eg(const double *epart, const int *ecount, const double *gpart, const int *gcount,
                            int stride, int k, double *out, hipStream_t st);
hipError_t launch_reduce_rows(const double *partial, const int *counts, int stride, int rows,
                              double scale, double *out, hipStream_t st);

hipError_t launch_gather(int precision, const void *psi, const uint64_t *Xa, const uint64_t *Xb,
                         const uint32_t *sa, const uint32_t *PPb, int64_t nsa, int64_t nsb,
                         double2 *C, hipStream_t st);
hipError_t launch_scatter(int precision, void *lam, const double2 *S, const uint64_t *Xa,
                          const uint64_t *Xb, const uint32_t *sa, const uint32_t *PPb,
                          int64_t nsa, int64_t nsb, hipStream_t st);
hipError_t launch_rdm_overlap(const double2 *A, int64_t nrows, int64_t ncols,
                              const uint32_t *exc, int nexc, double2 *O, hipStream_t st);
hipError_t launch_rdm_bin(const double2 *O, const int32_t *off, const int32_t *idx, int nbins,
                          double2 *out, hipStream_t st);

// ---- sector-compressed kernels (fsv_sigma.hip) ----
// Amplitude storage of a compact sector vector.
enum VType { V_C128 = 0, V_C64 = 1, V_F64 = 2, V_F32 = 3 };
inline int vtype_bytes(int vt) { return vt == V_C128 ? 16 : (vt == V_F32 ? 4 : 8); }

// Device tables of one sector Hamiltonian (alpha-first basis).
struct SectorTabs {
    int64_t nsa, nsb;
    int M, nexcA, nexcB;
    const int64_t *ha_ptr, *hb_ptr;
    const int32_t *ha_col, *hb_col;
    const double *ha_val, *hb_val;
    const uint32_t *excA, *excB;
    const uint32_t *excBT;  // excB transposed: [f][Ib]
    const double *g;
    double ecore;
    // Optional exact factorisation (pq|rs) = sum_l L[l][pq] L[l][rs] of rank R
    // (pivoted Cholesky of the pair supermatrix): Lt holds L transposed and
    // padded to RP = 8 columns (M^2 x RP, zero beyond R) and YT is an
    // RP * nsa * nsb work array (complex-sized).  R = 0 (also for every rank
    // above 8): direct product.
    int R;
    const double *Lt;
    void *YT;
    // Optional dense same-spin string Hamiltonians (nsa x nsa, nsb x nsb,
    // row-major) applied as FP64 GEMMs through the rocBLAS handle blas;
    // nullptr: the CSR rows above.
    const double *ha_dense, *hb_dense;
    void *blas;
    // hb_dense transposed (its column-major form): real states add the beta
    // product into S with one untransposed GEMM on it
    const double *hb_dense_t;
    // With the factorisation: per alpha (beta) string, the factor rows of its
    // diagonal excitations summed (nsa x RP, nsb x RP).  Each string's list in
    // excA / excB ends with its ndA (ndB) diagonal entries p -> p.
    const double *lr_da, *lr_db;
    int ndA, ndB;
};

int cadj_blocks(const PairOp &op, int64_t nsa, int64_t nsb);  // partials written by launch_cadj
hipError_t launch_crot(int vtype, void *psi, const PairOp &op, const uint32_t *lists,
                       const double *cs, int k, int64_t nsa, int64_t nsb, hipStream_t st);
hipError_t launch_cadj(int vtype, void *psi, void *lam, const PairOp &op, const uint32_t *lists,
                       const double *cs, int k, int64_t nsa, int64_t nsb, double *partial,
                       hipStream_t st);
// Real sector states (V_F64 / V_F32) only: z[i] = (psi[i], lam[i]) for i < n,
// and launch_cadj on such interleaved pairs.
hipError_t launch_zip(int vtype, const void *psi, const void *lam, void *z, int64_t n, hipStream_t st);
hipError_t launch_cadj_zip(int vtype, void *z, const PairOp &op, const uint32_t *lists, const double *cs, int k,
                           int64_t nsa, int64_t nsb, double *partial, hipStream_t st);
// out (vtype_out) <- in (vtype_in), element-wise; complex <-> real keeps the real part.
hipError_t launch_convert(int vt_in, const void *in, int vt_out, void *out, int64_t n, hipStream_t st);
// S = H C on the sector; C, S, CT, ST hold nsa*nsb values of type complex
// (cplex) or real double.  Writes combine_grid(nsa*nsb) partials of Re<C|S>.
// zout (real states, may be null): where the product's last step allows it,
// the (C, S) pairs go to zout instead of S, and *zipped is set.
unsigned combine_grid(int64_t dim);
// Whether the product on a real (cplex = false) or complex sector state writes
// the factorised intermediate YT (the two-kernel form of the alpha-beta term).
bool lr_uses_intermediate(const SectorTabs &T, bool cplex);
hipError_t launch_sector_sigma(bool cplex, const SectorTabs &T, const void *C, void *S, void *CT,
                               void *ST, double *epart, hipStream_t st, void *zout = nullptr,
                               bool *zipped = nullptr);
// ADAPT pool screening on a real sector state (V_F64 / V_F32): grid (gx, n_ops),
// partial[t * gx + x] = workgroup x's share of Re<lam|T_t|psi> for pool op t.
hipError_t launch_pool(int vtype, const void *psi, const void *lam, const PairOp *ops, const uint32_t *lists,
                       int n_ops, int gx, int64_t nsa, int64_t nsb, double *partial, hipStream_t st);
// String Hamiltonian values val[e] = v2[e] + one-body part of descriptor
// desc[e] with h~ = ht (M x M): -1 none, -2 - I the diagonal of row I (sum of
// h~_ii over the occupied orbitals of string str[I]), otherwise h~[desc &
// 0x3FFFFFFF], negated when bit 30 is set.
hipError_t launch_string_h_values(double *val, const double *v2, const int32_t *desc, const uint32_t *str,
                                  const double *ht, int M, int64_t n, hipStream_t st);
// Dense row-major copy (n x n) of an n-row CSR matrix.
hipError_t launch_csr_dense(const int64_t *rowptr, const int32_t *col, const double *val, double *out, int64_t n,
                            hipStream_t st);
// Transpose of a compact vector (rows x cols -> cols x rows), complex or real.
hipError_t launch_ctranspose(bool cplex, const void *in, void *out, int64_t rows, int64_t cols,
                             hipStream_t st);
// Real compact vector (double) -> dense complex buffer, like launch_scatter.
hipError_t launch_scatter_real(int precision, void *lam, const double *S, const uint64_t *Xa,
                               const uint64_t *Xb, const uint32_t *sa, const uint32_t *PPb,
                               int64_t nsa, int64_t nsb, hipStream_t st);
void init_sigma_kernels();

// ---- fused operator runs on the sector state (fsv_fused.hip, fsv_packet.hip) ----
constexpr int kPacketAmps = 256;  // amplitudes (index slots) of one packet
// A run of consecutive operators applied tile by tile in LDS (fused = 1), by
// connected-component packets (fused = 2), or a single operator left to the
// per-operator kernels (fused = 0, nops = 1).  A tile run keeps, per alpha
// orbit, a program of astride words (row count, row ranks, per-operator local
// alpha pairs) and, per beta block, one of bstride words (first column, width,
// per-operator local beta pairs).  A packet run keeps n_packets index lists
// (at ent_off, 256 words each) and regions of wr words (at reg_off).
struct FGroup {
    int32_t k0, nops, fused;
    int32_t n_orbits, n_blocks;  // tiles = n_orbits x n_blocks
    int32_t rmax, lmax;          // largest orbit (rows) and block (columns)
    int32_t astride, bstride;
    int64_t aprog_off, bprog_off;
    size_t lds;                  // dynamic LDS bytes of one tile / packet workgroup
    int32_t n_packets, wr;
    int64_t ent_off, reg_off;
    // Forward sweep from the reference state: while the state is zero outside
    // a few components, only the packets that hold nonzero amplitudes need to
    // run.  sub_n >= 0: those packets' programs, copied contiguously at
    // sub_ent_off / sub_reg_off; -1: launch every packet.
    int32_t sub_n = -1;
    int64_t sub_ent_off = 0, sub_reg_off = 0;
};

struct FusedOpts {
    size_t budget = 65536;       // LDS bytes of tile data per workgroup
    size_t lds_limit = 65536;    // dynamic LDS a workgroup may use
    int es = 8;                  // bytes per stored amplitude
    int arrays = 1;              // 1: forward (psi); 2: adjoint (psi and lam)
    int mode = 0;                // 0 fuse where the cost model gains, 1 never, 2 every run of >= 2
    int cus = 256;               // compute units (tiles resident at once scale with it)
    int min_block = 32;          // columns per block when blocks are split for more tiles
    int max_ops = 32;            // operators per run
    int64_t max_tiles = 8192;    // tiles per run (gradient partial slots per operator)
    bool place_xcd = true;       // packet runs: place components by XCD (padding with empty packets)
};

struct FusedSched {
    std::vector<FGroup> groups;  // in operator order
    std::vector<int> count;      // per operator: gradient partials of its fused run, -1 if not fused
    uint32_t *d_aprog = nullptr, *d_bprog = nullptr;  // packet runs: index lists, regions
    bool packets = false;        // built by build_packets: the adjoint sweep runs on (psi, lam) pairs
    std::vector<std::shared_ptr<void>> mem;  // device buffers (shared by schedules that alias them)
    size_t bytes = 0;                        // their size
    void release();
    void share(const FusedSched &o) {  // the same runs and device tables as o
        release();
        groups = o.groups;
        count = o.count;
        d_aprog = o.d_aprog;
        d_bprog = o.d_bprog;
        packets = o.packets;
        mem = o.mem;
        bytes = o.bytes;
    }
    FusedSched() = default;
    FusedSched(const FusedSched &) = delete;
    FusedSched &operator=(const FusedSched &) = delete;
    ~FusedSched() { release(); }
};

// Runs and tiles for the operators (K x 4 spin-orbital labels in ops, their
// pair ops and host pair lists) under o.  Returns an FSV_ status.
int build_fused(int M, const std::vector<uint32_t> &sa, const std::vector<uint32_t> &sb,
                const std::vector<PairOp> &pops, const std::vector<uint32_t> &lists,
                const std::vector<int32_t> &ops, const FusedOpts &o, FusedSched &S);
int fused_runs(const FusedSched &S, int *n_fused_ops);
// Host side of packet runs: groups (fused = 2 for packet runs, 0 for
// operators left alone), per-operator partial counts, and the index lists and
// regions (FGroup::ent_off / reg_off index ent / reg).  every_run: every run,
// a single operator's included, becomes a packet run.
struct PacketPlan {
    std::vector<FGroup> groups;
    std::vector<int> count;
    std::vector<uint32_t> ent, reg;
};
int plan_packets(int64_t nsa, int64_t nsb, const std::vector<PairOp> &pops, const std::vector<uint32_t> &lists,
                 const FusedOpts &o, bool every_run, PacketPlan &S);
// Batched packet runs over independent instances (real FP64 states in one
// arena): launch r carries run r - (R - runs_i) of every instance i (runs
// aligned at the end, so the adjoint sweep runs the same launches backwards).
struct BatchPacketInst {
    int64_t nsa, nsb, off_state, off_ops, off_k;
    int32_t K;
};
struct BatchPackets {
    int runs = 0;
    int pstride = 1;                       // gradient partial slots per operator
    std::vector<int64_t> ent_off, reg_off;  // per launch
    std::vector<int32_t> wr, npk;           // per launch: region stride, packets
    std::vector<uint32_t> ent, reg;
    std::vector<int32_t> count;             // per operator (global index): partials of its run
};
int build_batch_packets(const std::vector<BatchPacketInst> &insts, const std::vector<PairOp> &ops,
                        const std::vector<uint32_t> &lists, BatchPackets &B);
size_t batch_packet_lds(int wr, bool adjoint);
hipError_t launch_batch_packets(bool adjoint, double *arena, const uint32_t *ent, const uint32_t *reg, int wr,
                                int npk, const double *cs, double *gpart, int pstride, hipStream_t st);

// Packet runs (fused = 2) for sector states of at most packet_max_dim()
// amplitudes; o.es, o.mode (0 cost model, 1 never, otherwise every run of >= 2)
// and o.max_ops are used.  count[k] = gradient partials of operator k's run.
// Plans use them by default up to packet_default_dim() amplitudes (above it
// only on request: planning time and program memory grow with the state).
int64_t packet_max_dim();
int64_t packet_default_dim();
int build_packets(int64_t nsa, int64_t nsb, const std::vector<PairOp> &pops, const std::vector<uint32_t> &lists,
                  const FusedOpts &o, FusedSched &S);
// One packet run: forward (state = psi) or adjoint (state = the interleaved
// (psi, lam) pairs of launch_zip; gradient partials gpart[k * gstride + workgroup]).
// t0, t1 (optional): events given the kernel's own start and end times.
// store = false: the run's results are not written back (nothing reads them:
// the adjoint sweep's last run).
hipError_t launch_packets(int vtype, bool adjoint, void *state, const FusedSched &S, const FGroup &g,
                          const double *cs, double *gpart, int gstride, hipStream_t st, hipEvent_t t0 = nullptr,
                          hipEvent_t t1 = nullptr, bool store = true);
void init_fused_kernels();
size_t fused_lds_limit();
// Forward (psi) or adjoint (psi, lam, gradient partials gpart[k * gstride + tile]).
// Packet groups are launched with launch_packets.
hipError_t launch_fused(int vtype, bool adjoint, void *psi, void *lam, const FusedSched &S, const FGroup &g,
                        const PairOp *d_pops, const double *cs, int64_t nsb, double *gpart, int gstride,
                        hipStream_t st);

}  // namespace fsv
