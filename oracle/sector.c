/*
 * Sector-compressed FP64 CPU oracle (test infrastructure only; never part of
 * the product path).
 *
 * What it computes, from the paper's definitions:
 *  - Fermionic operators act on Jordan-Wigner qubit strings (one spin-orbital
 *    per qubit, Introduction; the JW mapping of a^+ a, Strategy 2 density
 *    matrix paragraph).  a_q |x> = (-1)^popcount(x & (2^q - 1)) |x ^ 2^q> when
 *    bit q is set, else 0; a^+_q likewise with bit q clear.  Every sign below is
 *    obtained by applying the operators one at a time in this way.
 *  - Excitation rotations U = exp(theta (tau - tau^+)), tau = a^+_a a^+_b a_j a_i
 *    (singles a^+_a a_i); U acts on the pairs (x, x') with tau|x> = s|x'>.
 *    Excitation kind 1 (qubit excitations, the QEB pool of the paper's ADAPT
 *    runs, Computational Details) applies the same factors as qubit raising /
 *    lowering operators: the bit flips without a parity sign.
 *  - ADAPT pool screening: for each pool operator the energy derivative of
 *    appending it at angle 0, <psi|[H, T]|psi> = 2 Re <H psi| T |psi>.
 *  - The Hamiltonian with the Strategy-2 one-body potential folded into h:
 *      H = E_core + sum_{pq,s} h_pq a^+_{ps} a_{qs}
 *             + 1/2 sum_{pqrs,st} (pq|rs) a^+_{ps} a^+_{rt} a_{st} a_{qs}
 *    with spatial-orbital chemist-notation integrals (FCIDUMP convention,
 *    Computational Details).
 *  - The one-particle density matrix n_{pq,s} = <psi| a^+_{ps} a_{qs} |psi>
 *    (Strategy 2 density matrix equation).
 *
 * Only the (N_alpha, N_beta) sector is stored: the operators above conserve
 * both electron counts, so every amplitude outside that sector of a state built
 * from the reference determinant is exactly zero.  Sector element r = Ia*nsb+Ib
 * holds the amplitude of the qubit string x = X_alpha[Ia] | X_beta[Ib] in the
 * plan's qubit ordering (0: qubit 2p+s, 1: qubit p+s*M).
 *
 * For the Hamiltonian the amplitudes are first rewritten in the alpha-string-
 * first product form |Ia>|Ib> (a permutation sign counted pair by pair); in
 * that form the alpha-beta two-body term is sum (pq|rs) E^a_pq E^b_rs and the
 * same-spin terms act on one string alone.  Both string-space operators are
 * built by applying the literal operator strings to every string.
 *
 * Arrays: complex values are interleaved (re, im) doubles.  Functions return 0
 * on success, a negative value on bad arguments or allocation failure.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int M, na, nb, ordering;
    long nsa, nsb, dim;
    uint32_t *sa, *sb;      /* orbital bitmasks, ascending */
    int32_t *ranka, *rankb; /* 2^M lookup, -1 when not in list */
    uint64_t *xa, *xb;      /* qubit string of each alpha / beta string */
    int qa[32], qb[32];     /* qubit of orbital p for each spin */
    int exc;                /* excitation kind: 0 fermionic, 1 qubit */
} sec_t;

static int popc64(uint64_t v) { return __builtin_popcountll(v); }

static int qubit_of(int M, int ordering, int p, int s) {
    return ordering == 0 ? 2 * p + s : p + s * M;
}

/* Apply a^+_q (dag=1) or a_q (dag=0) to the string *x in place.  Returns the
 * JW sign (+1/-1) or 0 when the operator annihilates the string.  qubit = 1:
 * the qubit raising / lowering operator instead (sign +1). */
static int jw(uint64_t *x, int dag, int q, int qubit) {
    uint64_t bit = 1ull << q;
    if (dag) {
        if (*x & bit) return 0;
    } else {
        if (!(*x & bit)) return 0;
    }
    int par = qubit ? 0 : (popc64(*x & (bit - 1)) & 1);
    *x ^= bit;
    return par ? -1 : 1;
}

static void sec_free(sec_t *S) {
    free(S->sa); free(S->sb); free(S->ranka); free(S->rankb); free(S->xa); free(S->xb);
    memset(S, 0, sizeof(*S));
}

static long binom(int n, int k) {
    if (k < 0 || k > n) return 0;
    long r = 1;
    for (int i = 1; i <= k; ++i) r = r * (n - k + i) / i;
    return r;
}

static int make_strings(int M, int ne, uint32_t **out, int32_t **rank, long *count) {
    long cnt = binom(M, ne);
    uint32_t *s = (uint32_t *)malloc(sizeof(uint32_t) * (cnt > 0 ? cnt : 1));
    int32_t *rk = (int32_t *)malloc(sizeof(int32_t) * (1u << M));
    if (!s || !rk) { free(s); free(rk); return -2; }
    long c = 0;
    for (uint32_t m = 0; m < (1u << M); ++m) {
        if (__builtin_popcount(m) == ne) { rk[m] = (int32_t)c; s[c++] = m; }
        else rk[m] = -1;
    }
    *out = s; *rank = rk; *count = c;
    return 0;
}

static int sec_init(sec_t *S, int M, int na, int nb, int ordering) {
    memset(S, 0, sizeof(*S));
    if (M < 1 || M > 17 || na < 0 || nb < 0 || na > M || nb > M || (ordering != 0 && ordering != 1))
        return -1;
    S->M = M; S->na = na; S->nb = nb; S->ordering = ordering;
    if (make_strings(M, na, &S->sa, &S->ranka, &S->nsa)) { sec_free(S); return -2; }
    if (make_strings(M, nb, &S->sb, &S->rankb, &S->nsb)) { sec_free(S); return -2; }
    S->dim = S->nsa * S->nsb;
    for (int p = 0; p < M; ++p) { S->qa[p] = qubit_of(M, ordering, p, 0); S->qb[p] = qubit_of(M, ordering, p, 1); }
    S->xa = (uint64_t *)malloc(sizeof(uint64_t) * S->nsa);
    S->xb = (uint64_t *)malloc(sizeof(uint64_t) * S->nsb);
    if (!S->xa || !S->xb) { sec_free(S); return -2; }
    for (long i = 0; i < S->nsa; ++i) {
        uint64_t x = 0;
        for (int p = 0; p < M; ++p) if (S->sa[i] >> p & 1u) x |= 1ull << S->qa[p];
        S->xa[i] = x;
    }
    for (long i = 0; i < S->nsb; ++i) {
        uint64_t x = 0;
        for (int p = 0; p < M; ++p) if (S->sb[i] >> p & 1u) x |= 1ull << S->qb[p];
        S->xb[i] = x;
    }
    return 0;
}

/* Sector index of a qubit string, or -1 when it lies outside the sector. */
static long sec_index(const sec_t *S, uint64_t x) {
    uint32_t a = 0, b = 0;
    for (int p = 0; p < S->M; ++p) {
        a |= (uint32_t)((x >> S->qa[p]) & 1u) << p;
        b |= (uint32_t)((x >> S->qb[p]) & 1u) << p;
    }
    int32_t ia = S->ranka[a], ib = S->rankb[b];
    if (ia < 0 || ib < 0) return -1;
    return (long)ia * S->nsb + ib;
}

/* tau = a^+_a a^+_b a_j a_i (op = {a, b, j, i}; singles have b = j = -1).
 * adjoint = 1 applies tau^+ = a^+_i a^+_j a_b a_a instead. */
static int apply_tau(const sec_t *S, const int32_t *op, int adjoint, uint64_t *x) {
    int q[4], d[4], cnt = 0;
    int a = op[0], b = op[1], j = op[2], i = op[3];
#define SOQ(so) qubit_of(S->M, S->ordering, (so) / 2, (so) % 2)
    if (!adjoint) {
        q[cnt] = SOQ(i); d[cnt++] = 0;
        if (j >= 0) { q[cnt] = SOQ(j); d[cnt++] = 0; }
        if (b >= 0) { q[cnt] = SOQ(b); d[cnt++] = 1; }
        q[cnt] = SOQ(a); d[cnt++] = 1;
    } else {
        q[cnt] = SOQ(a); d[cnt++] = 0;
        if (b >= 0) { q[cnt] = SOQ(b); d[cnt++] = 0; }
        if (j >= 0) { q[cnt] = SOQ(j); d[cnt++] = 1; }
        q[cnt] = SOQ(i); d[cnt++] = 1;
    }
#undef SOQ
    int sign = 1;
    for (int k = 0; k < cnt; ++k) {
        int s = jw(x, d[k], q[k], S->exc);
        if (!s) return 0;
        sign *= s;
    }
    return sign;
}

static int check_ops(int M, int K, const int32_t *ops) {
    int n = 2 * M;
    for (int k = 0; k < K; ++k) {
        const int32_t *o = ops + 4 * k;
        int single = (o[1] < 0);
        if (single && o[2] >= 0) return -1;
        if (!single && o[2] < 0) return -1;
        if (o[0] < 0 || o[0] >= n || o[3] < 0 || o[3] >= n) return -1;
        if (!single && (o[1] >= n || o[2] >= n)) return -1;
    }
    return 0;
}

/* psi <- U(theta) psi for one excitation operator, pair by pair. */
static void rotate(const sec_t *S, const int32_t *op, double theta, double *psi) {
    const double c = cos(theta), sn = sin(theta);
    const long dim = S->dim, nsb = S->nsb;
#pragma omp parallel for schedule(static)
    for (long r = 0; r < dim; ++r) {
        uint64_t x = S->xa[r / nsb] | S->xb[r % nsb];
        int s = apply_tau(S, op, 0, &x);
        if (!s) continue;
        long rp = sec_index(S, x);
        if (rp < 0) continue; /* cannot happen for spin-conserving ops */
        double ar = psi[2 * r], ai = psi[2 * r + 1];
        double br = psi[2 * rp], bi = psi[2 * rp + 1];
        psi[2 * r] = c * ar - s * sn * br;
        psi[2 * r + 1] = c * ai - s * sn * bi;
        psi[2 * rp] = c * br + s * sn * ar;
        psi[2 * rp + 1] = c * bi + s * sn * ai;
    }
}

long or_dim(int M, int na, int nb) { return binom(M, na) * binom(M, nb); }

/* Dense qubit-string index of every sector element, in sector order. */
int or_sector_qubit_index(int M, int na, int nb, int ordering, uint64_t *xout) {
    sec_t S;
    int rc = sec_init(&S, M, na, nb, ordering);
    if (rc) return rc;
    for (long r = 0; r < S.dim; ++r) xout[r] = S.xa[r / S.nsb] | S.xb[r % S.nsb];
    sec_free(&S);
    return 0;
}

static void set_reference(const sec_t *S, double *psi) {
    memset(psi, 0, sizeof(double) * 2 * S->dim);
    long ia = S->ranka[(1u << S->na) - 1], ib = S->rankb[(1u << S->nb) - 1];
    psi[2 * (ia * S->nsb + ib)] = 1.0;
}

/* psi = U_K(theta_K) ... U_1(theta_1) |reference>; first listed op first. */
int or_ansatz(int M, int na, int nb, int ordering, int K, const int32_t *ops,
              const double *theta, int excitation, double *psi) {
    sec_t S;
    if (check_ops(M, K, ops)) return -1;
    int rc = sec_init(&S, M, na, nb, ordering);
    if (rc) return rc;
    S.exc = excitation;
    set_reference(&S, psi);
    for (int k = 0; k < K; ++k) rotate(&S, ops + 4 * k, theta[k], psi);
    sec_free(&S);
    return 0;
}

/* Apply the listed rotations in order to a given sector vector. */
int or_apply_rotations(int M, int na, int nb, int ordering, int K, const int32_t *ops,
                       const double *theta, int excitation, double *psi) {
    sec_t S;
    if (check_ops(M, K, ops)) return -1;
    int rc = sec_init(&S, M, na, nb, ordering);
    if (rc) return rc;
    S.exc = excitation;
    for (int k = 0; k < K; ++k) rotate(&S, ops + 4 * k, theta[k], psi);
    sec_free(&S);
    return 0;
}

/* ---------------- Hamiltonian in the alpha-first string product form ---------- */

typedef struct { int32_t J; int16_t p, q; int8_t s; } exc_t;

typedef struct {
    long ns;
    long *off;      /* CSR row offsets (gather form: row I lists J with <I|op|J> != 0) */
    exc_t *e;
} exclist_t;

typedef struct {
    long ns;
    long *off;
    int32_t *col;
    double *val;
} csr_t;

/* Single-excitation lists E_pq |J> = s |I>, stored by output string I. */
static int build_exc(int M, const uint32_t *str, const int32_t *rank, long ns, exclist_t *L) {
    long *cnt = (long *)calloc(ns + 1, sizeof(long));
    if (!cnt) return -2;
    for (long J = 0; J < ns; ++J)
        for (int p = 0; p < M; ++p)
            for (int q = 0; q < M; ++q) {
                uint64_t x = str[J];
                int s = jw(&x, 0, q, 0);
                if (!s) continue;
                int s2 = jw(&x, 1, p, 0);
                if (!s2) continue;
                cnt[rank[x] + 1]++;
            }
    for (long I = 0; I < ns; ++I) cnt[I + 1] += cnt[I];
    exc_t *e = (exc_t *)malloc(sizeof(exc_t) * (cnt[ns] > 0 ? cnt[ns] : 1));
    long *fill = (long *)calloc(ns, sizeof(long));
    if (!e || !fill) { free(cnt); free(e); free(fill); return -2; }
    for (long J = 0; J < ns; ++J)
        for (int p = 0; p < M; ++p)
            for (int q = 0; q < M; ++q) {
                uint64_t x = str[J];
                int s = jw(&x, 0, q, 0);
                if (!s) continue;
                int s2 = jw(&x, 1, p, 0);
                if (!s2) continue;
                long I = rank[x];
                exc_t t = {(int32_t)J, (int16_t)p, (int16_t)q, (int8_t)(s * s2)};
                e[cnt[I] + fill[I]++] = t;
            }
    free(fill);
    L->ns = ns; L->off = cnt; L->e = e;
    return 0;
}

/* Same-spin string Hamiltonian: sum_pq h_pq a^+_p a_q + 1/2 sum_pqrs (pq|rs)
 * a^+_p a^+_r a_s a_q acting on one spin's strings.  Built column by column by
 * applying each operator string to each string J, then compressed by rows. */
static int build_same_spin(int M, const uint32_t *str, const int32_t *rank, long ns,
                           const double *h, const double *g, csr_t *H) {
    double *dense = (double *)calloc((size_t)ns * ns, sizeof(double));
    if (!dense) return -2;
    const long M2 = (long)M * M, M3 = M2 * M;
#pragma omp parallel for schedule(dynamic, 4)
    for (long J = 0; J < ns; ++J) {
        for (int p = 0; p < M; ++p)
            for (int q = 0; q < M; ++q) {
                uint64_t x = str[J];
                int s = jw(&x, 0, q, 0);
                if (!s) continue;
                int s2 = jw(&x, 1, p, 0);
                if (!s2) continue;
                dense[(size_t)rank[x] * ns + J] += h[p * M + q] * s * s2;
            }
        /* a^+_p a^+_r a_s a_q: a_q acts first, then a_s, a^+_r, a^+_p */
        for (int q = 0; q < M; ++q) {
            uint64_t x1 = str[J];
            int t1 = jw(&x1, 0, q, 0);
            if (!t1) continue;
            for (int s_ = 0; s_ < M; ++s_) {
                uint64_t x2 = x1;
                int t2 = jw(&x2, 0, s_, 0);
                if (!t2) continue;
                for (int r = 0; r < M; ++r) {
                    uint64_t x3 = x2;
                    int t3 = jw(&x3, 1, r, 0);
                    if (!t3) continue;
                    for (int p = 0; p < M; ++p) {
                        uint64_t x4 = x3;
                        int t4 = jw(&x4, 1, p, 0);
                        if (!t4) continue;
                        double v = 0.5 * g[p * M3 + q * M2 + r * M + s_];
                        dense[(size_t)rank[x4] * ns + J] += v * t1 * t2 * t3 * t4;
                    }
                }
            }
        }
    }
    long *off = (long *)calloc(ns + 1, sizeof(long));
    if (!off) { free(dense); return -2; }
    for (long I = 0; I < ns; ++I) {
        long c = 0;
        for (long J = 0; J < ns; ++J) c += dense[(size_t)I * ns + J] != 0.0;
        off[I + 1] = off[I] + c;
    }
    int32_t *col = (int32_t *)malloc(sizeof(int32_t) * (off[ns] > 0 ? off[ns] : 1));
    double *val = (double *)malloc(sizeof(double) * (off[ns] > 0 ? off[ns] : 1));
    if (!col || !val) { free(dense); free(off); free(col); free(val); return -2; }
    for (long I = 0; I < ns; ++I) {
        long k = off[I];
        for (long J = 0; J < ns; ++J) {
            double v = dense[(size_t)I * ns + J];
            if (v != 0.0) { col[k] = (int32_t)J; val[k] = v; ++k; }
        }
    }
    free(dense);
    H->ns = ns; H->off = off; H->col = col; H->val = val;
    return 0;
}

/* Permutation sign between the qubit-ordered product of creators and the
 * alpha-first product: (-1)^{#(beta r, alpha q) occupied with qubit(beta r) <
 * qubit(alpha q)}, counted pair by pair. */
static int order_sign(const sec_t *S, long ia, long ib) {
    int cnt = 0;
    for (int q = 0; q < S->M; ++q) {
        if (!(S->sa[ia] >> q & 1u)) continue;
        for (int r = 0; r < S->M; ++r)
            if ((S->sb[ib] >> r & 1u) && S->qb[r] < S->qa[q]) ++cnt;
    }
    return (cnt & 1) ? -1 : 1;
}

int or_sigma(int M, int na, int nb, int ordering, const double *h, const double *g,
             double e_core, const double *psi, double *sig) {
    sec_t S;
    int rc = sec_init(&S, M, na, nb, ordering);
    if (rc) return rc;
    const long nsa = S.nsa, nsb = S.nsb, dim = S.dim;
    const long M2 = (long)M * M;
    double *c = (double *)malloc(sizeof(double) * 2 * dim);
    double *out = (double *)calloc(2 * dim, sizeof(double));
    int8_t *phi = (int8_t *)malloc(dim);
    exclist_t La = {0}, Lb = {0};
    csr_t Ha = {0}, Hb = {0};
    if (!c || !out || !phi) { rc = -2; goto done; }
#pragma omp parallel for schedule(static)
    for (long r = 0; r < dim; ++r) {
        phi[r] = (int8_t)order_sign(&S, r / nsb, r % nsb);
        c[2 * r] = phi[r] * psi[2 * r];
        c[2 * r + 1] = phi[r] * psi[2 * r + 1];
    }
    if ((rc = build_exc(M, S.sa, S.ranka, nsa, &La))) goto done;
    if ((rc = build_exc(M, S.sb, S.rankb, nsb, &Lb))) goto done;
    if ((rc = build_same_spin(M, S.sa, S.ranka, nsa, h, g, &Ha))) goto done;
    if ((rc = build_same_spin(M, S.sb, S.rankb, nsb, h, g, &Hb))) goto done;

#pragma omp parallel for schedule(dynamic, 1)
    for (long Ia = 0; Ia < nsa; ++Ia) {
        double *o = out + 2 * Ia * nsb;
        /* alpha-alpha: sum_Ja Ha[Ia][Ja] c[Ja][:] */
        for (long k = Ha.off[Ia]; k < Ha.off[Ia + 1]; ++k) {
            const double v = Ha.val[k];
            const double *cj = c + 2 * (long)Ha.col[k] * nsb;
            for (long Ib = 0; Ib < nsb; ++Ib) {
                o[2 * Ib] += v * cj[2 * Ib];
                o[2 * Ib + 1] += v * cj[2 * Ib + 1];
            }
        }
        /* beta-beta: sum_Jb Hb[Ib][Jb] c[Ia][Jb] */
        const double *ci = c + 2 * Ia * nsb;
        for (long Ib = 0; Ib < nsb; ++Ib)
            for (long k = Hb.off[Ib]; k < Hb.off[Ib + 1]; ++k) {
                o[2 * Ib] += Hb.val[k] * ci[2 * Hb.col[k]];
                o[2 * Ib + 1] += Hb.val[k] * ci[2 * Hb.col[k] + 1];
            }
        /* alpha-beta: sum (pq|rs) E^a_pq E^b_rs */
        for (long ka = La.off[Ia]; ka < La.off[Ia + 1]; ++ka) {
            const exc_t ea = La.e[ka];
            const double *gpq = g + (ea.p * M + ea.q) * M2;
            const double *cj = c + 2 * (long)ea.J * nsb;
            for (long Ib = 0; Ib < nsb; ++Ib) {
                double ar = 0.0, ai = 0.0;
                for (long kb = Lb.off[Ib]; kb < Lb.off[Ib + 1]; ++kb) {
                    const exc_t eb = Lb.e[kb];
                    const double w = gpq[eb.p * M + eb.q] * eb.s;
                    ar += w * cj[2 * eb.J];
                    ai += w * cj[2 * eb.J + 1];
                }
                o[2 * Ib] += ea.s * ar;
                o[2 * Ib + 1] += ea.s * ai;
            }
        }
        for (long Ib = 0; Ib < nsb; ++Ib) {
            o[2 * Ib] += e_core * ci[2 * Ib];
            o[2 * Ib + 1] += e_core * ci[2 * Ib + 1];
        }
    }
#pragma omp parallel for schedule(static)
    for (long r = 0; r < dim; ++r) {
        sig[2 * r] = phi[r] * out[2 * r];
        sig[2 * r + 1] = phi[r] * out[2 * r + 1];
    }
done:
    free(c); free(out); free(phi);
    free(La.off); free(La.e); free(Lb.off); free(Lb.e);
    free(Ha.off); free(Ha.col); free(Ha.val); free(Hb.off); free(Hb.col); free(Hb.val);
    sec_free(&S);
    return rc;
}

/* gamma[s][p][q] = <psi| a^+_{ps} a_{qs} |psi>, complex, 2*M*M*2 doubles. */
int or_rdm1(int M, int na, int nb, int ordering, const double *psi, double *gamma) {
    sec_t S;
    int rc = sec_init(&S, M, na, nb, ordering);
    if (rc) return rc;
    const long dim = S.dim, nsb = S.nsb;
    memset(gamma, 0, sizeof(double) * 4 * M * M);
    for (int s = 0; s < 2; ++s)
        for (int p = 0; p < M; ++p)
            for (int q = 0; q < M; ++q) {
                const int qp = qubit_of(M, ordering, p, s), qq = qubit_of(M, ordering, q, s);
                double re = 0.0, im = 0.0;
#pragma omp parallel for reduction(+ : re, im) schedule(static)
                for (long r = 0; r < dim; ++r) {
                    uint64_t x = S.xa[r / nsb] | S.xb[r % nsb];
                    int t1 = jw(&x, 0, qq, 0);
                    if (!t1) continue;
                    int t2 = jw(&x, 1, qp, 0);
                    if (!t2) continue;
                    long rp = sec_index(&S, x);
                    /* conj(psi[rp]) * sign * psi[r] */
                    double sr = psi[2 * rp], si = psi[2 * rp + 1];
                    double vr = psi[2 * r], vi = psi[2 * r + 1];
                    re += t1 * t2 * (sr * vr + si * vi);
                    im += t1 * t2 * (sr * vi - si * vr);
                }
                gamma[((s * M + p) * M + q) * 2] = re;
                gamma[((s * M + p) * M + q) * 2 + 1] = im;
            }
    sec_free(&S);
    return 0;
}

/* <lam| T |psi> with T = tau - tau^+, evaluated by applying tau and tau^+ to
 * every sector string.  Returns the real part (the imaginary part of the
 * overlap is not needed for the gradient 2 Re<lam|T|psi>). */
static double overlap_T(const sec_t *S, const int32_t *op, const double *lam, const double *psi) {
    const long dim = S->dim, nsb = S->nsb;
    double acc = 0.0;
#pragma omp parallel for reduction(+ : acc) schedule(static)
    for (long r = 0; r < dim; ++r) {
        for (int adj = 0; adj < 2; ++adj) {
            uint64_t x = S->xa[r / nsb] | S->xb[r % nsb];
            int s = apply_tau(S, op, adj, &x);
            if (!s) continue;
            long rp = sec_index(S, x);
            double w = adj ? -s : s;
            /* Re(conj(lam[rp]) * w * psi[r]) */
            acc += w * (lam[2 * rp] * psi[2 * r] + lam[2 * rp + 1] * psi[2 * r + 1]);
        }
    }
    return acc;
}

/*
 * Energy and gradient by the adjoint method with stored forward states:
 *   psi_k = U_k ... U_1 psi_0 (psi_0 = |ref>, or the given initial sector
 *   vector), lam_k = U_{k+1}^+ ... U_K^+ H psi_K,
 *   dE/dtheta_k = 2 Re <lam_k| T_k |psi_k>.
 * The states before operators 0, stride, 2*stride, ... are kept; each
 * segment's intermediate states are recomputed forward once from its kept
 * state when the reverse pass reaches it (stride = 1 recomputes one operator).
 */
int or_energy_grad(int M, int na, int nb, int ordering, const double *h, const double *g,
                   double e_core, int K, const int32_t *ops, const double *theta, int excitation,
                   const double *psi0, int stride, double *E, double *grad) {
    sec_t S;
    if (check_ops(M, K, ops)) return -1;
    if (stride < 1) stride = 1;
    int rc = sec_init(&S, M, na, nb, ordering);
    if (rc) return rc;
    S.exc = excitation;
    const long dim = S.dim;
    const size_t vb = sizeof(double) * 2 * dim;
    const int nstore = K / stride + 1;
    double **store = (double **)calloc(nstore, sizeof(double *));
    double *psi = (double *)malloc(vb), *lam = (double *)malloc(vb);
    double *seg = NULL;
    if (!store || !psi || !lam) { rc = -2; goto done; }
    for (int i = 0; i < nstore; ++i) {
        store[i] = (double *)malloc(vb);
        if (!store[i]) { rc = -2; goto done; }
    }
    if (psi0) memcpy(psi, psi0, vb); /* a given initial state instead of |ref> */
    else set_reference(&S, psi);
    for (int k = 0; k < K; ++k) {
        if (k % stride == 0) memcpy(store[k / stride], psi, vb);
        rotate(&S, ops + 4 * k, theta[k], psi);
    }
    /* psi now = psi_K */
    rc = or_sigma(M, na, nb, ordering, h, g, e_core, psi, lam);
    if (rc) goto done;
    {
        double e = 0.0;
        for (long r = 0; r < dim; ++r) e += psi[2 * r] * lam[2 * r] + psi[2 * r + 1] * lam[2 * r + 1];
        *E = e;
    }
    /* Segments [b, e) of `stride` operators, last segment first: the states
     * after operators b..e-1 are recomputed once from checkpoint b, then the
     * segment's gradients are taken in reverse order. */
    seg = (double *)malloc(vb * (size_t)stride);
    if (!seg) { rc = -2; goto done; }
    for (int i = (K - 1) / stride; K > 0 && i >= 0; --i) {
        const int b = i * stride, e = (b + stride < K) ? b + stride : K;
        memcpy(seg, store[i], vb);
        rotate(&S, ops + 4 * b, theta[b], seg);
        for (int t = b + 1; t < e; ++t) {
            double *dst = seg + (size_t)(t - b) * 2 * dim;
            memcpy(dst, dst - 2 * dim, vb);
            rotate(&S, ops + 4 * t, theta[t], dst);
        }
        for (int k = e - 1; k >= b; --k) {
            const double *pk = seg + (size_t)(k - b) * 2 * dim; /* state after operator k */
            grad[k] = 2.0 * overlap_T(&S, ops + 4 * k, lam, pk);
            rotate(&S, ops + 4 * k, -theta[k], lam);
        }
    }
done:
    if (store) for (int i = 0; i < nstore; ++i) free(store[i]);
    free(store); free(psi); free(lam); free(seg);
    sec_free(&S);
    return rc;
}

/* ADAPT screening: grad[t] = 2 Re <H psi| T_t |psi> for the P pool operators
 * (kind `excitation`) at the sector state psi. */
int or_pool_gradients(int M, int na, int nb, int ordering, const double *h, const double *g,
                      double e_core, const double *psi, int P, const int32_t *pool, int excitation,
                      double *grad) {
    sec_t S;
    if (check_ops(M, P, pool)) return -1;
    int rc = sec_init(&S, M, na, nb, ordering);
    if (rc) return rc;
    S.exc = excitation;
    double *lam = (double *)malloc(sizeof(double) * 2 * S.dim);
    if (!lam) { sec_free(&S); return -2; }
    rc = or_sigma(M, na, nb, ordering, h, g, e_core, psi, lam);
    if (!rc)
        for (int t = 0; t < P; ++t) grad[t] = 2.0 * overlap_T(&S, pool + 4 * t, lam, psi);
    free(lam);
    sec_free(&S);
    return rc;
}

int or_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
