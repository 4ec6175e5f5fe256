/*
 * fsv.h -- fermionic state-vector emulation on one AMD MI355X (gfx950).
 *
 * The GPU side of the hybrid scheme of arXiv 2405.11567 (Fig. 1: the QPU
 * workload replaced by a GPU emulator): a variational fermionic ansatz on a
 * 2^n complex amplitude vector, its energy <H> for a second-quantised
 * Hamiltonian given by one- and two-electron integrals (exchanged as FCIDUMP
 * integrals, Computational Details), the one-particle density matrix of
 * Strategy 2, and the extra one-body potential that the self-consistent
 * Strategy-2 loop adds to the Hamiltonian (effective Hamiltonian equation).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - n_qubits = 2 * n_orb.  Spin-orbital label so = 2 p + s (s = 0 alpha,
 *    s = 1 beta).  The qubit holding so is so for ordering 0 (interleaved) and
 *    p + s * n_orb for ordering 1 (blocked).  Bit j of a basis index x is the
 *    occupation of qubit j, and |x> = prod_{j ascending} (a^+_j)^{x_j} |vac>
 *    (Jordan-Wigner mapping, one spin-orbital per qubit).
 *  - An operator is four int32 {a, b, j, i}: tau = a^+_a a^+_b a_j a_i; a
 *    single excitation is {a, -1, -1, i}: tau = a^+_a a_i.  Indices are
 *    spin-orbital labels; they must be distinct, in range and conserve the
 *    number of alpha and of beta electrons.  With excitation = 1 the same four
 *    labels name a qubit excitation (the factors act as qubit raising /
 *    lowering operators, without JW signs).  U_k = exp(theta_k (tau - tau^+)),
 *    theta in radians, and the ansatz is U_K ... U_1 |ref>: the first listed
 *    operator acts first.  |ref> fills the lowest n_alpha alpha and n_beta beta
 *    orbitals with amplitude +1 (the paper's HF initial state).
 *  - H = e_core + sum_{pq,s} (h + v)_pq a^+_{ps} a_{qs}
 *          + 1/2 sum_{pqrs,st} (pq|rs) a^+_{ps} a^+_{rt} a_{st} a_{qs},
 *    h: n_orb x n_orb real symmetric, row-major; g: n_orb^4 real, row-major,
 *    chemist notation (pq|rs) with 8-fold symmetry; v: the Strategy-2 one-body
 *    potential (zero until set_onebody_potential is called).
 *  - Amplitude buffers are device pointers to 2^n complex values: interleaved
 *    (re, im) float64 for precision 0, float32 for precision 1.  The caller
 *    owns and allocates them (fsv_state_bytes); the library never allocates
 *    O(2^n) memory.
 *  - Device memory of a plan (all of it sized by the (n_alpha, n_beta)
 *    sector, the only part of the state the operators above ever make
 *    nonzero, of dimension D = C(n_orb, n_alpha) C(n_orb, n_beta)):
 *      - its tables, owned by the plan and allocated at creation: operator pair
 *        lists, string tables and same-spin string Hamiltonians (sparse rows,
 *        and dense copies of D_alpha^2 + 2 D_beta^2 doubles where the dense
 *        products are chosen), integrals, and the programs of the fused
 *        operator runs (fsv_plan_runs); fsv_plan_device_bytes reports them;
 *      - its workspace of fsv_plan_workspace_bytes: four complex sector
 *        vectors (16 D bytes each), the factorised alpha-beta intermediate
 *        (8 x 16 D bytes, when that product is used), density-matrix overlaps
 *        and the per-operator gradient partials (K x 8192 doubles).  The caller
 *        may provide it (fsv_plan_set_workspace; the Python binding allocates
 *        it through PyTorch, so that running out of memory shows up there);
 *        otherwise the plan allocates it on the first call that needs it.
 *    The FP64 GEMM library used for dense same-spin products keeps its own
 *    small per-handle workspace besides.
 *  - Every function returns FSV_OK (0) or a negative status, never throws and
 *    never exits.  fsv_last_error() returns a thread-local message for the last
 *    failure on the calling thread.
 *  - A plan is bound to the HIP stream given at creation (NULL: the legacy
 *    default stream).  Work is ordered after all earlier work on that stream;
 *    functions that write host outputs return after the results are on the
 *    host.  A plan is not thread-safe: calls on one plan must not overlap.
 */
#ifndef FSV_H
#define FSV_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FSV_OK 0
#define FSV_EINVAL -1     /* invalid argument: index, size, ordering, precision, symmetry */
#define FSV_ENOMEM -2     /* plan tables could not be allocated (host or device) */
#define FSV_EDEVICE -3    /* HIP runtime error; the message holds the HIP error string */
#define FSV_ESTATE -4     /* wrong call order or a plan / batch mismatch */
#define FSV_ENONFINITE -5 /* NaN or Inf in theta, h, g or v */

typedef struct fsv_plan fsv_plan;
typedef struct fsv_batch fsv_batch;
typedef struct fsv_pool fsv_pool;

typedef struct {
    int32_t n_qubits;   /* 2 .. 34, even */
    int32_t n_alpha;    /* 0 .. n_orb */
    int32_t n_beta;     /* 0 .. n_orb */
    int32_t ordering;   /* 0 interleaved (qubit 2p+s), 1 blocked (qubit p + s*n_orb) */
    int32_t precision;  /* 0 complex128 amplitudes, 1 complex64 amplitudes (FP64 reductions) */
    const double *h;    /* host, n_orb*n_orb, copied at plan creation */
    const double *g;    /* host, n_orb^4, copied at plan creation */
    double e_core;      /* constant added through H (0 for synthetic inputs) */
    int32_t n_ops;      /* K >= 0 */
    const int32_t *ops; /* host, K x 4 {a, b, j, i}, copied at plan creation */
    int32_t excitation; /* 0 fermionic excitations (JW signs); 1 qubit excitations
                           (QEB: Q^+_a Q^+_b Q_j Q_i on the plan's qubits, every
                           pair sign +1 in the qubit basis; the pool of the
                           paper's ADAPT runs, Computational Details) */
} fsv_problem;

/* Message of the last failure on this thread ("" when none). */
const char *fsv_last_error(void);

/* Build a plan: validate the problem, compile each operator into bit masks,
 * build the alpha/beta string tables of the sector and upload the integrals.
 * hip_stream is a hipStream_t (NULL allowed).  On failure *out is NULL. */
int fsv_plan_create(fsv_plan **out, const fsv_problem *problem, void *hip_stream);

/* Release a plan and its device tables.  NULL is accepted. */
int fsv_plan_destroy(fsv_plan *plan);

/* Bytes of one amplitude buffer: 2^n_qubits * (16 or 8). 0 for NULL. */
size_t fsv_state_bytes(const fsv_plan *plan);

/* Bytes of the plan's workspace (see the conventions above).  0 for NULL. */
size_t fsv_plan_workspace_bytes(const fsv_plan *plan);

/* Device bytes the plan owns now: its tables, plus its workspace when the
 * plan allocated that itself.  0 for NULL. */
size_t fsv_plan_device_bytes(const fsv_plan *plan);

/* Give the plan a caller-owned workspace: ws_dev (device, 256-byte aligned)
 * of at least fsv_plan_workspace_bytes bytes, which the caller keeps alive
 * and unused by other work until the plan is destroyed or another workspace
 * is set.  A workspace the plan allocated itself is freed.  ws_dev = NULL
 * goes back to a plan-owned workspace (allocated on the next call).  Waits
 * for the plan's earlier work.  Its contents between calls are unspecified.
 * Errors: FSV_EINVAL (NULL plan, too small or misaligned), FSV_EDEVICE. */
int fsv_plan_set_workspace(fsv_plan *plan, void *ws_dev, size_t bytes);

/* Sector dimensions: number of alpha strings, beta strings, and the dense
 * index of the reference determinant.  Any pointer may be NULL. */
int fsv_plan_info(const fsv_plan *plan, int64_t *n_alpha_strings, int64_t *n_beta_strings,
                  uint64_t *reference_index);

/* Choose how energy_grad, energy_grad_fd and the stage calls hold the state:
 * 0 (default) keeps only the (n_alpha, n_beta) sector, compactly, in the first
 * C(n_orb, n_alpha) * C(n_orb, n_beta) amplitudes of the work buffers (every
 * other amplitude of a state built from |ref> is exactly zero, since each
 * operator conserves both electron counts); 1 uses the full 2^n layout and
 * touches every active amplitude pair of each operator.  Results agree to
 * rounding.  The environment variable FSV_ENGINE=dense selects 1 at creation. */
int fsv_plan_set_engine(fsv_plan *plan, int engine);

/* Operator runs of the sector engine's forward sweep (adjoint = 0) or adjoint
 * sweep (adjoint = 1).  Each rotation exp(theta (tau - tau^+)) mixes only
 * the two amplitudes of each of its active pairs, so consecutive operators can
 * be applied together in one launch:
 *  - component packets (the default for sector states of at most 2^22
 *    amplitudes; FSV_FUSE=packets requests them up to 2^26, where every run
 *    becomes a packet run: at 30 qubits an evaluation takes 71 instead of
 *    83 ms, but planning takes ~3 minutes and the programs 13 GB of device
 *    memory; FSV_VERBOSE prints a line per planned run): the connected components of the graph joining the amplitudes
 *    that some operator of the run pairs are mutually independent; runs are
 *    extended while every component has at most 256 amplitudes, and whole
 *    components are packed into 256-amplitude packets, one wavefront each;
 *  - LDS tiles (larger states, FSV_FUSE=tiles): tiles that the whole run maps
 *    onto themselves (alpha strings that agree outside the run's alpha
 *    orbitals x a block of beta strings), chosen from an LDS budget.
 * A cost model decides which runs are fused (FSV_NO_FUSE: none,
 * FSV_FORCE_FUSE: every tile run of two or more); fsv_autotune retunes.
 * run_start[k] receives the first operator of the run holding operator k,
 * fused_tiles[k] the tiles or packets of its fused launch, or 0 when k is
 * applied alone (host arrays of K int32, either may be NULL).  Returns the
 * number of runs (>= 0) or a negative status. */
int fsv_plan_runs(const fsv_plan *plan, int adjoint, int32_t *run_start, int32_t *fused_tiles);

/* Profiling: the sector engine's forward sweep (adjoint = 0: psi is
 * initialised, then every run) or adjoint sweep (adjoint = 1: psi and lam must
 * hold the final state and H psi, as after fsv_forward_async and
 * fsv_sigma_async; the runs are applied last to first and the gradient is
 * reduced into the plan's output, readable with fsv_finish) launched without a
 * graph.  A packet run's time is its kernel's own duration (events given the
 * kernel's start and end); any other run's is the time between events recorded
 * around its launches.  ms (host, one float per run of fsv_plan_runs, operator
 * order) receives each run's time in milliseconds.
 * Synchronises the plan's stream.  Returns the number of runs (>= 0), or -1
 * for NULL arguments, -4 on the dense engine, -3 on a HIP error. */
int fsv_time_runs(fsv_plan *plan, int adjoint, void *psi_dev, void *lam_dev, float *ms);

/* psi_dev <- U_K(theta_K) ... U_1(theta_1) |ref> (ansatz preparation on the
 * GPU emulator, Fig. 1).  theta: host, K doubles.  Every amplitude of psi_dev
 * is written (zero outside the sector). */
int ansatz_apply(fsv_plan *plan, const double *theta, void *psi_dev);

/* *E_out <- Re <psi| H |psi> for the (n_alpha, n_beta) sector component of
 * psi, without normalisation (the expectation value <H> of Fig. 1; the
 * Strategy-1 input).  psi_dev is read only. */
int energy(fsv_plan *plan, const void *psi_dev, double *E_out);

/* Energy of psi(theta) and its gradient dE/dtheta_k by the adjoint method:
 * after the forward sweep lam = H psi, then for k = K..1
 * grad_k = 2 Re <lam| (tau_k - tau_k^+) |psi>, psi <- U_k^+ psi,
 * lam <- U_k^+ lam (the states are recomputed, never stored).  psi_dev and
 * lam_dev are caller-owned work buffers of fsv_state_bytes each; their
 * contents on return are unspecified.  grad_out: host, K doubles. */
int energy_grad(fsv_plan *plan, const double *theta, void *psi_dev, void *lam_dev,
                double *E_out, double *grad_out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * energy and adjoint gradient as energy_grad (same kernels, same results to
 * rounding), with no allocation in the call.  Its per-call scratch (the
 * interleaved (psi, lam) pairs of the adjoint sweep, the transposes and the
 * factorised intermediate of H psi, the energy and gradient partials) lives in
 * one static device block of 64 MiB per GPU that the library holds until the
 * process ends, not in the plan's workspace.  A plan whose scratch exceeds the
 * block (sector states above roughly 1.3 M amplitudes at K = 200) gets
 * FSV_EINVAL, the needed size in the message; the dense engine gets
 * FSV_ESTATE.  Kernels are launched one by one (no graph is captured or
 * instantiated).  Every call on one GPU shares its block: calls that overlap
 * on one GPU (plans on different streams, or threads) race and must be
 * serialised by the caller.  Nothing in the block needs to start at zero; its
 * contents between calls are unspecified.  Arguments as for energy_grad. */
int energy_grad_noalloc(fsv_plan *plan, const double *theta, void *psi_dev, void *lam_dev, double *E_out,
                        double *grad_out);

/* Same energy and gradient by central finite differences of the energy,
 * 2K + 1 energy evaluations with step `step` (the plain per-parameter method
 * the adjoint is compared against).  psi_dev is a work buffer. */
int energy_grad_fd(fsv_plan *plan, const double *theta, double step, void *psi_dev,
                   double *E_out, double *grad_out);

/* One-particle density matrix gamma[s][p][q] = <psi| a^+_{ps} a_{qs} |psi>
 * (Strategy 2, density-matrix equation) for s = alpha, beta.  gamma_out: host,
 * 2 * n_orb * n_orb complex128 as interleaved doubles (4 n_orb^2 doubles). */
int rdm1(fsv_plan *plan, const void *psi_dev, double *gamma_out);

/* Replace the one-body potential: the Hamiltonian becomes H with h -> h + v
 * (the basis-set correction potential operator of Strategy 2, spin-independent).
 * v: host, n_orb*n_orb real symmetric (row-major, copied; the caller keeps
 * ownership); NULL clears it.  The string Hamiltonian tables are refreshed on
 * the device from their fixed two-body parts; the call waits for the plan's
 * earlier work first.  Captured graphs read the tables, so later energy,
 * energy_grad, stage-level and pool calls on this plan use the new
 * Hamiltonian without re-capture (batches hold their own Hamiltonians).
 * Errors: FSV_EINVAL (NULL plan, v not symmetric to 1e-12 of its largest
 * entry), FSV_ENONFINITE (NaN or Inf in v); the old potential stays then. */
int set_onebody_potential(fsv_plan *plan, const double *v);

/* ---- stage-level asynchronous entry points (device outputs, no host sync) ----
 * They split energy_grad into its passes so that a caller can time or overlap
 * them; energy_grad is exactly forward + sigma + reverse + finish. */

/* Upload theta (host, K) into the plan's device angle table. */
int fsv_set_theta(fsv_plan *plan, const double *theta);
/* psi <- |ref>, then the K forward rotations with the uploaded angles. */
int fsv_forward_async(fsv_plan *plan, void *psi_dev);
/* lam <- H psi (zero outside the sector); E on the device. */
int fsv_sigma_async(fsv_plan *plan, const void *psi_dev, void *lam_dev);
/* Reverse adjoint sweep over all K operators (psi = the forward sweep's
 * result, lam = H psi); per-operator partial sums on the device.  The contents
 * of psi_dev and lam_dev on return are unspecified. */
int fsv_reverse_async(fsv_plan *plan, void *psi_dev, void *lam_dev);
/* Reduce the partial sums, copy E and grad to the host and wait. */
int fsv_finish(fsv_plan *plan, double *E_out, double *grad_out);

/* Autotuner.  Sector engine: time whole energy + gradient evaluations for
 * candidate LDS budgets of the fused operator runs (and for one launch per
 * operator) and keep the fastest.  Dense engine: time the rotation and adjoint
 * kernels over candidate launch shapes and keep the fastest (cached per shape
 * class in the file named by FSV_TUNE_CACHE when set).  psi_dev and lam_dev
 * are distinct work buffers.  *report (may be NULL) receives a static summary
 * string. */
int fsv_autotune(fsv_plan *plan, void *psi_dev, void *lam_dev, const char **report);

/* Start the ansatz from a multi-determinant state instead of |ref> (the
 * paper warm-starts its runs from CIPSI wavefunctions, Computational
 * Details): sum_d coef[d] |dets[d]>, dets = qubit strings (host, n_det
 * uint64; bit j = qubit j in the plan's ordering), each in the
 * (n_alpha, n_beta) sector and listed once; coef: host, n_det real values,
 * used as given (not normalised).  n_det = 0 restores |ref>.  Later
 * ansatz_apply, energy_grad, energy_grad_fd, the stage calls and pools start
 * from it (captured graphs are rebuilt).  Errors: FSV_EINVAL (a determinant
 * outside the sector, repeated, or with bits above the last qubit),
 * FSV_ENONFINITE, FSV_ENOMEM. */
int fsv_set_initial_state(fsv_plan *plan, int32_t n_det, const uint64_t *dets, const double *coef);

/* First-order property <psi| D |psi> of a spin-independent one-body operator
 * D = sum_{pq,s} d_pq a^+_{ps} a_{qs} (e.g. a dipole component with d the
 * dipole integrals, evaluated from the Strategy-2 density as tr(d gamma)):
 * out[0] + i out[1] = sum_pq d_pq (gamma_alpha + gamma_beta)_pq, from the
 * 1-RDM of psi_dev (read only).  d: host, n_orb x n_orb real, row-major, need
 * not be symmetric.  out: host, 2 doubles. */
int onebody_expectation(fsv_plan *plan, const void *psi_dev, const double *d, double *out);

/* ---- ADAPT operator-pool screening ----
 * ADAPT grows the ansatz by the pool operator with the largest energy
 * derivative (Computational Details: ADAPT-VQE with a QEB pool).  For an
 * operator T appended at angle 0 to the plan's ansatz at theta that
 * derivative is <psi| [H, T] |psi> = 2 Re <H psi| T |psi>, psi = psi(theta).
 * fsv_pool_create compiles a pool for a plan (which must use the sector
 * engine): ops is host, n_ops x 4 {a, b, j, i} in the plan's conventions,
 * excitation 0 fermionic / 1 qubit (as in fsv_problem).  Pools and plans may
 * be destroyed in either order: a pool whose plan is gone can still be
 * destroyed, and fsv_pool_gradients on it returns FSV_ESTATE.
 * Errors: FSV_EINVAL for an invalid operator, FSV_ESTATE for a dense-engine
 * plan, FSV_ENOMEM, FSV_EDEVICE. */
int fsv_pool_create(fsv_pool **out, fsv_plan *plan, const int32_t *ops, int32_t n_ops, int32_t excitation);
int fsv_pool_destroy(fsv_pool *pool);
/* Prepare psi(theta), lam = H psi, then screen every pool operator in one
 * launch: grad_out[t] = 2 Re <lam| T_t |psi> (host, n_ops doubles); *E_out
 * (may be NULL) receives E(theta).  theta: host, K doubles of the plan.
 * psi_dev and lam_dev are distinct work buffers of fsv_state_bytes each. */
int fsv_pool_gradients(fsv_pool *pool, const double *theta, void *psi_dev, void *lam_dev, double *E_out,
                       double *grad_out);

/* ---- batches: many independent instances in one graph launch ----
 * Each instance has its own problem (qubit count, electrons, integrals,
 * operators; at most 24 qubits: larger systems belong in a plan); all must use
 * precision 0.  Real angles and integrals keep every amplitude real, so each
 * instance's sector state psi and its H psi are stored as real FP64 in a
 * device arena of fsv_batch_arena_bytes that the caller owns and passes to
 * every evaluation (the batch owns only its tables, fsv_batch_bytes).  H C: for instances of at least 16 x 16 strings the
 * same-spin part runs as dense FP64 products on the matrix cores (all such
 * instances in one launch; FSV_BATCH_SAME_SPIN=sparse keeps them on sparse
 * rows), then one workgroup per (instance, alpha string) adds the rest with
 * the row staged in LDS (the alpha-beta term through exact low-rank factors of
 * (pq|rs) where they exist, FSV_BATCH_SIGMA=direct avoids them; rows too long
 * for the LDS budget, or FSV_BATCH_SIGMA=global, read global memory only).
 * Three launch schemes, chosen by fsv_batch_autotune (or FSV_BATCH_MODE =
 * packets | phased | persistent at creation), each captured into one graph
 * that a call launches once: component-packet runs (the default when every
 * instance has at most 2^22 sector amplitudes; launch r carries run r of
 * every instance, runs aligned at their ends, so the graph holds two
 * launches per run index plus the H psi and reduction launches, about 33 for
 * 256 instances of 50..150 operators); phased launches (one per operator
 * index and phase, every instance in each); or a single persistent kernel
 * whose workgroups take whole instances from a device work queue, largest
 * first (measured slower than packet runs on that workload, so not the
 * default).  Results are identical to rounding.  Errors: FSV_EINVAL for an
 * invalid instance (the message names it), FSV_ENOMEM, FSV_EDEVICE. */
int fsv_batch_create(fsv_batch **out, const fsv_problem *problems, int32_t count, void *hip_stream);
int fsv_batch_destroy(fsv_batch *batch);
/* Bytes of the state arena an evaluation needs: 2 x 8 x sum_i D_i (psi and
 * H psi of every instance, real FP64).  0 for NULL. */
size_t fsv_batch_arena_bytes(const fsv_batch *batch);
/* theta_concat: host, sum_i K_i doubles in instance order.  arena_dev:
 * device, 256-byte aligned, at least fsv_batch_arena_bytes bytes, owned by
 * the caller; its contents on return are unspecified (a different arena than
 * the previous call's makes the batch capture its graph again).  E_out: host,
 * count doubles.  grad_concat: host, sum_i K_i doubles.  Errors: FSV_EINVAL
 * (NULL or misaligned arguments), FSV_ENONFINITE, FSV_EDEVICE. */
int fsv_batch_energy_grad(fsv_batch *batch, const double *theta_concat, void *arena_dev, double *E_out,
                          double *grad_concat);
/* Device bytes the batch owns (its tables and initial-state lists; the arena
 * is the caller's). */
size_t fsv_batch_bytes(const fsv_batch *batch);
/* Start instance `instance` (0-based) from a multi-determinant state instead
 * of its reference determinant (the paper warm-starts from CIPSI
 * wavefunctions, Computational Details): sum_d coef[d] |dets[d]>, dets = qubit
 * strings (host, n_det uint64; bit j = qubit j in that instance's ordering),
 * each in the instance's (n_alpha, n_beta) sector and listed once; coef:
 * host, n_det real values, used as given.  n_det = 0 restores the reference
 * determinant.  Every launch scheme starts that instance from the list on
 * later evaluations (the captured graph is rebuilt).  The lists are batch
 * tables (counted by fsv_batch_bytes).  Errors: FSV_EINVAL (instance out of
 * range; a determinant outside the sector, repeated, or with bits above the
 * instance's last qubit), FSV_ENONFINITE, FSV_ENOMEM, FSV_EDEVICE. */
int fsv_batch_set_initial_state(fsv_batch *batch, int32_t instance, int32_t n_det, const uint64_t *dets,
                                const double *coef);
/* Autotuner: times every candidate on this batch through its own captured
 * graph and keeps the fastest: launch scheme, persistent workgroup size and
 * workgroups per CU, phased workgroups per instance, and the LDS budget of an
 * H C workgroup (which sets how many alpha excitations it stages per pass).
 * arena_dev as for fsv_batch_energy_grad.  *report (may be NULL) receives a
 * static summary string. */
int fsv_batch_autotune(fsv_batch *batch, void *arena_dev, const char **report);

#ifdef __cplusplus
}
#endif

#endif /* FSV_H */
