// Fused runs of excitation rotations on the sector state C[Ia][Ib] (real,
// FP64 or FP32 storage).
//
// An excitation changes occupations only inside the orbitals it names, so a
// run of consecutive operators whose alpha parts together name the alpha
// orbitals S_a and whose beta parts name S_b maps each tile
//     (alpha strings that agree outside S_a)  x  (beta strings that agree on
//      the top b orbitals, none of which is in S_b)
// onto itself.  Strings are ranked in ascending bit-mask order, so a beta
// block is a contiguous range of columns and every tile row is a contiguous
// segment of one C row.  One workgroup per tile first copies the tile's
// program (its row ranks, column range and, per operator, the alpha and beta
// pairs in tile-local coordinates, all precomputed on the host) and the run's
// angles into LDS, then the tile itself; it applies the whole run there with
// LDS reads only (forward: rotations in order; adjoint: for k = last..first
// the gradient partial of operator k, then psi and lam un-rotated) and writes
// the tile back: one pass over the state per run, with two dependent rounds of
// global loads, instead of one launch per operator.  Runs and tiles are chosen
// on the host from an LDS budget, the number of tiles the chip holds at once
// and a simple cost model (runs of small, latency-bound operators are fused;
// runs whose tiles would move far more bytes than their operators' active
// pairs are not).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <vector>

#include "fsv_device.h"
#include "fsv_internal.h"

namespace fsv {

namespace {

constexpr int kMaxTileRows = 255;  // local row indices are packed in 8 bits
constexpr int kMaxTileCols = 32767;  // local column indices are packed in 15 bits
constexpr int kFusedBlock = 512;
constexpr int kBatch = 8;  // global loads in flight per thread while a tile is staged
constexpr uint32_t kAll = 0xFFFFFFFFu;  // pair count of an operator without a part on this spin

// Program layouts (32-bit words).
//   orbit:  [0] nr, [1 .. 1+rmax) row ranks, [1+rmax+2j] offset and
//           [2+rmax+2j] count of operator j's local alpha pairs
//           (src | dst << 8 | neg << 31), then the pairs.
//   block:  [0] first column, [1] width L, [2+2j] offset and [3+2j] count of
//           operator j's local beta pairs (src | dst << 15 | neg << 31).
struct FArgs {
    int32_t k0, nops, n_blocks, gstride;
    int32_t astride, bstride, rmax, lmax;
    int64_t nsb;
    const uint32_t *aprog, *bprog;  // this run's programs
    const PairOp *ops;
    const double *cs;
};

template <typename T>
__device__ __forceinline__ void rotT(T &a, T &b, T c, T s) {
    const T t = a;
    a = c * a - s * b;
    b = c * b + s * t;
}

template <typename T, bool ADJ>
__global__ __launch_bounds__(kFusedBlock) void k_fused(T *__restrict__ psi, T *__restrict__ lam, FArgs a,
                                                      double *__restrict__ gpart) {
    extern __shared__ double lds[];
    const int tsz = a.rmax * a.lmax;
    double *scs = lds;                               // 2 nops angles (cos, sin)
    T *tp = (T *)(lds + 2 * a.nops);                 // psi tile
    T *tl = tp + tsz;                                // lam tile (adjoint)
    uint32_t *pa = (uint32_t *)(tp + (ADJ ? 2 : 1) * tsz);
    uint32_t *pb = pa + a.astride;
    int32_t *sg0 = (int32_t *)(pb + a.bstride);
    const int tile = blockIdx.x;
    const int o = tile / a.n_blocks, b = tile - o * a.n_blocks;
    // first loads: programs, angles, operator signs.  Indices are clamped rather
    // than branched on so that each thread's loads are all in flight before
    // the first LDS write.
    {
        const uint32_t *ga = a.aprog + (int64_t)o * a.astride, *gb = a.bprog + (int64_t)b * a.bstride;
        const int tot = a.astride + a.bstride;
        const int tc = min((int)threadIdx.x, 2 * a.nops - 1), ts = min((int)threadIdx.x, a.nops - 1);
        const double vcs = a.cs[2 * a.k0 + tc];
        const int32_t vsg = a.ops[a.k0 + ts].sign0;
        for (int base = 0; base < tot; base += kBatch * kFusedBlock) {
            uint32_t v[kBatch];
#pragma unroll
            for (int m = 0; m < kBatch; ++m) {
                const int i = min(base + m * kFusedBlock + (int)threadIdx.x, tot - 1);
                v[m] = *(i < a.astride ? ga + i : gb + (i - a.astride));
            }
#pragma unroll
            for (int m = 0; m < kBatch; ++m) {
                const int i = base + m * kFusedBlock + (int)threadIdx.x;
                if (i < tot) pa[i] = v[m];  // pb follows pa directly
            }
        }
        if ((int)threadIdx.x < 2 * a.nops) scs[threadIdx.x] = vcs;
        if ((int)threadIdx.x < a.nops) sg0[threadIdx.x] = vsg;
    }
    __syncthreads();
    const int nr = (int)pa[0], L = (int)pb[1];
    const int64_t c0 = pb[0];
    const uint32_t *rows = pa + 1;
    const int n = nr * L;
    // second loads: the tile, kBatch loads per thread in flight
    for (int base = 0; base < n; base += kBatch * kFusedBlock) {
        T v[kBatch], w[kBatch];
#pragma unroll
        for (int m = 0; m < kBatch; ++m) {
            const int i = min(base + m * kFusedBlock + (int)threadIdx.x, n - 1);
            const int r = i / L, c = i - r * L;
            const int64_t x = (int64_t)rows[r] * a.nsb + c0 + c;
            v[m] = psi[x];
            if (ADJ) w[m] = lam[x];
        }
#pragma unroll
        for (int m = 0; m < kBatch; ++m) {
            const int i = base + m * kFusedBlock + (int)threadIdx.x;
            if (i < n) {
                tp[i] = v[m];
                if (ADJ) tl[i] = w[m];
            }
        }
    }
    __syncthreads();
    for (int jj = 0; jj < a.nops; ++jj) {
        const int j = ADJ ? a.nops - 1 - jj : jj;
        const T c = (T)scs[2 * j], s = (T)scs[2 * j + 1];
        const uint32_t aoff = pa[1 + a.rmax + 2 * j], acnt = pa[2 + a.rmax + 2 * j];
        const uint32_t boff = pb[2 + 2 * j], bcnt = pb[3 + 2 * j];
        const int na = acnt == kAll ? nr : (int)acnt, nb = bcnt == kAll ? L : (int)bcnt;
        const bool neg0 = sg0[j] < 0;
        const int nw = na * nb;
        double acc = 0.0;
        for (int w = threadIdx.x; w < nw; w += blockDim.x) {
            const int u = w / nb, v = w - u * nb;
            int ra = u, ra2 = u, cb = v, cb2 = v;
            bool neg = neg0;
            if (acnt != kAll) {
                const uint32_t e = pa[aoff + u];
                ra = (int)(e & 0xFFu);
                ra2 = (int)((e >> 8) & 0xFFu);
                neg ^= (e >> 31) != 0;
            }
            if (bcnt != kAll) {
                const uint32_t e = pb[boff + v];
                cb = (int)(e & 0x7FFFu);
                cb2 = (int)((e >> 15) & 0x7FFFu);
                neg ^= (e >> 31) != 0;
            }
            const int xs = ra * L + cb, xd = ra2 * L + cb2;
            T va = tp[xs], vb = tp[xd];
            if (ADJ) {
                T la = tl[xs], lb = tl[xd];
                const double ov = (double)lb * (double)va - (double)la * (double)vb;
                acc += neg ? -ov : ov;
                const T sg = neg ? s : -s;  // U^+ = U(-theta)
                rotT(va, vb, c, sg);
                rotT(la, lb, c, sg);
                tl[xs] = la;
                tl[xd] = lb;
            } else {
                rotT(va, vb, c, neg ? -s : s);
            }
            tp[xs] = va;
            tp[xd] = vb;
        }
        if (ADJ) {
            acc = block_sum(acc);  // its barriers also order operator j before the next
            if (threadIdx.x == 0) gpart[(int64_t)(a.k0 + j) * a.gstride + tile] = acc;
        } else {
            __syncthreads();
        }
    }
#pragma unroll 4
    for (int i = threadIdx.x; i < n; i += kFusedBlock) {
        const int r = i / L, c = i - r * L;
        const int64_t x = (int64_t)rows[r] * a.nsb + c0 + c;
        psi[x] = tp[i];
        if (ADJ) lam[x] = tl[i];
    }
}

// ---- host: tiles of a set of touched orbitals ----
struct TilePlan {
    bool ok = false;
    int bsplit = 0;  // top beta orbitals fixed per block
    int rmax = 0, lmax = 0;
    int64_t n_orbits = 0, n_blocks = 0, rounds = 0;
};

struct Planner {
    int M;
    const std::vector<uint32_t> &sa, &sb;
    std::vector<int32_t> cnt;  // scratch, 2^M
    Planner(int M_, const std::vector<uint32_t> &a, const std::vector<uint32_t> &b)
        : M(M_), sa(a), sb(b), cnt((size_t)1 << M_, 0) {}

    // largest orbit and number of orbits of the alpha strings under S_a
    void orbits(uint32_t Sa, int &rmax, int64_t &norb) {
        rmax = 0;
        norb = 0;
        for (uint32_t s : sa) {
            int &c = cnt[s & ~Sa];
            if (c == 0) ++norb;
            rmax = std::max(rmax, ++c);
        }
        for (uint32_t s : sa) cnt[s & ~Sa] = 0;
    }
    // column blocks when the top b beta orbitals are fixed
    void blocks(int b, int &lmax, int64_t &nblk) {
        lmax = 0;
        nblk = 0;
        int run = 0;
        uint32_t key = ~0u;
        for (uint32_t s : sb) {
            const uint32_t k2 = b ? (s >> (M - b)) : 0u;
            if (k2 != key) {
                key = k2;
                ++nblk;
                run = 0;
            }
            lmax = std::max(lmax, ++run);
        }
    }
    // Smallest number of rounds of resident tiles (ties: more, smaller tiles)
    // over the column splits whose tiles fit the budget.
    TilePlan fit(uint32_t Sa, uint32_t Sb, const FusedOpts &o) {
        TilePlan best;
        int rmax;
        int64_t norb;
        orbits(Sa, rmax, norb);
        if (rmax > kMaxTileRows || sa.empty() || sb.empty()) return best;
        const size_t per = (size_t)o.es * o.arrays;
        int bmax = 0;  // top beta orbitals outside S_b
        while (bmax < M && !((Sb >> (M - 1 - bmax)) & 1u)) ++bmax;
        bool first = true;
        for (int b = 0; b <= bmax; ++b) {
            int lmax;
            int64_t nblk;
            blocks(b, lmax, nblk);
            const size_t tile = (size_t)rmax * lmax * per;
            if (tile > o.budget || lmax > kMaxTileCols) continue;
            if (!first && lmax < o.min_block) break;
            first = false;
            const int64_t tiles = norb * nblk;
            if (tiles > o.max_tiles) break;
            // workgroups per CU: LDS (tile plus ~1/4 for programs), at most 4
            // of kFusedBlock threads
            const int64_t per_cu = std::max<int64_t>(1, std::min<int64_t>(4, 163840 / (tile + tile / 4 + 256)));
            const int64_t rounds = (tiles + o.cus * per_cu - 1) / (o.cus * per_cu);
            if (!best.ok || rounds <= best.rounds) {
                best.ok = true;
                best.bsplit = b;
                best.rmax = rmax;
                best.lmax = lmax;
                best.n_orbits = norb;
                best.n_blocks = nblk;
                best.rounds = rounds;
            }
        }
        return best;
    }
};

uint32_t spin_mask(const int32_t *op, int spin) {
    uint32_t m = 0;
    for (int t = 0; t < 4; ++t)
        if (op[t] >= 0 && op[t] % 2 == spin) m |= 1u << (op[t] / 2);
    return m;
}

}  // namespace

void FusedSched::release() {
    mem.clear();
    bytes = 0;
    groups.clear();
    count.clear();
    d_aprog = d_bprog = nullptr;
    packets = false;
}

int build_fused(int M, const std::vector<uint32_t> &sa, const std::vector<uint32_t> &sb,
                const std::vector<PairOp> &pops, const std::vector<uint32_t> &lists,
                const std::vector<int32_t> &ops, const FusedOpts &o, FusedSched &S) {
    S.release();
    const int K = (int)pops.size();
    S.count.assign(K, -1);
    if (K == 0) return FSV_OK;
    Planner pl(M, sa, sb);
    const int64_t nsa = (int64_t)sa.size(), nsb = (int64_t)sb.size();
    auto pairs_of = [&](const PairOp &p) {
        return (double)(p.nA >= 0 ? p.nA : nsa) * (double)(p.nB >= 0 ? p.nB : nsb);
    };
    // cost model (measured on MI355X at 24 qubits): a per-operator launch costs
    // ~3.5 us (forward) / ~5 us (adjoint) plus its active pairs' bytes at
    // ~4 TB/s; a fused run ~3.5 us of launch and program fetch per round of
    // resident tiles, ~0.6 us of LDS work per operator, and its whole-state
    // tile traffic at ~2 TB/s (latency-bound: the state is fetched in one round)
    const double bw = 4.0e12, bw_tile = 2.0e12;
    const double t_launch = o.arrays == 1 ? 3.5e-6 : 5.0e-6, t_round = 3.5e-6, t_op = 0.6e-6;
    const double bytes_amp = (double)o.es * o.arrays;

    std::vector<uint32_t> aprog, bprog;
    std::vector<int32_t> orb_of(nsa), loc(nsa), blk_of(nsb);
    std::vector<int32_t> first((size_t)1 << M, -1);
    auto single = [&](int k) {
        FGroup s{};
        s.k0 = k;
        s.nops = 1;
        S.groups.push_back(s);
    };
    int i = 0;
    while (i < K) {
        uint32_t Sa = spin_mask(&ops[4 * i], 0), Sb = spin_mask(&ops[4 * i], 1);
        TilePlan tp = o.mode == 1 ? TilePlan{} : pl.fit(Sa, Sb, o);
        int j = i + 1;
        if (tp.ok) {
            while (j < K && j - i < o.max_ops) {
                const uint32_t Sa2 = Sa | spin_mask(&ops[4 * j], 0), Sb2 = Sb | spin_mask(&ops[4 * j], 1);
                const TilePlan t2 = pl.fit(Sa2, Sb2, o);
                if (!t2.ok) break;
                Sa = Sa2;
                Sb = Sb2;
                tp = t2;
                ++j;
            }
        }
        const int nops = j - i;
        bool fuse = tp.ok && nops >= 2;
        if (fuse && o.mode == 0) {
            double t_ops = 0.0;
            for (int k = i; k < j; ++k) t_ops += t_launch + pairs_of(pops[k]) * 4.0 * bytes_amp / bw;
            const double t_f = (double)tp.rounds * t_round + nops * t_op +
                                (double)nsa * nsb * 2.0 * bytes_amp / bw_tile;
            fuse = t_f < t_ops;
        }
        if (!fuse) {
            for (int k = i; k < j; ++k) single(k);
            i = j;
            continue;
        }
        FGroup g{};
        g.k0 = i;
        g.nops = nops;
        g.fused = 1;
        g.rmax = tp.rmax;
        g.lmax = tp.lmax;
        g.n_orbits = (int32_t)tp.n_orbits;
        g.n_blocks = (int32_t)tp.n_blocks;
        // orbits in order of their smallest rank; local index = position in the orbit
        std::vector<std::vector<int32_t>> members;
        for (int64_t r = 0; r < nsa; ++r) {
            const uint32_t key = sa[r] & ~Sa;
            if (first[key] < 0) {
                first[key] = (int32_t)members.size();
                members.emplace_back();
            }
            orb_of[r] = first[key];
            loc[r] = (int32_t)members[first[key]].size();
            members[first[key]].push_back((int32_t)r);
        }
        for (int64_t r = 0; r < nsa; ++r) first[sa[r] & ~Sa] = -1;
        // column blocks: runs of equal top-b beta orbitals
        std::vector<int2> blocks;
        {
            const int b = tp.bsplit;
            uint32_t key = ~0u;
            for (int64_t c = 0; c < nsb; ++c) {
                const uint32_t k2 = b ? (sb[c] >> (M - b)) : 0u;
                if (k2 != key) {
                    key = k2;
                    blocks.push_back(make_int2((int)c, 0));
                }
                blocks.back().y += 1;
                blk_of[c] = (int32_t)blocks.size() - 1;
            }
        }
        // per-orbit alpha programs
        std::vector<std::vector<uint32_t>> ap(g.n_orbits);
        for (int32_t ob = 0; ob < g.n_orbits; ++ob) {
            std::vector<uint32_t> &w = ap[ob];
            w.assign(1 + g.rmax + 2 * nops, 0u);
            w[0] = (uint32_t)members[ob].size();
            for (size_t t = 0; t < members[ob].size(); ++t) w[1 + t] = (uint32_t)members[ob][t];
        }
        std::vector<std::vector<uint32_t>> bp(g.n_blocks);
        for (int32_t bk = 0; bk < g.n_blocks; ++bk) {
            std::vector<uint32_t> &w = bp[bk];
            w.assign(2 + 2 * nops, 0u);
            w[0] = (uint32_t)blocks[bk].x;
            w[1] = (uint32_t)blocks[bk].y;
        }
        for (int jj = 0; jj < nops; ++jj) {
            const PairOp &p = pops[i + jj];
            const int ha = 1 + g.rmax + 2 * jj, hb = 2 + 2 * jj;
            if (p.nA < 0) {
                for (auto &w : ap) w[ha + 1] = kAll;
            } else {
                std::vector<std::vector<uint32_t>> per(g.n_orbits);
                for (int32_t u = 0; u < p.nA; ++u) {
                    const uint32_t e = lists[p.offA + u];
                    const int32_t s = (int32_t)(e & 0x7FFFu), d = (int32_t)((e >> 15) & 0x7FFFu);
                    if (orb_of[s] != orb_of[d])
                        return fail(FSV_EINVAL, "internal: alpha pair leaves its orbit (operator %d)", i + jj);
                    per[orb_of[s]].push_back((uint32_t)loc[s] | ((uint32_t)loc[d] << 8) | (e & 0x80000000u));
                }
                for (int32_t ob = 0; ob < g.n_orbits; ++ob) {
                    std::vector<uint32_t> &w = ap[ob];
                    w[ha] = (uint32_t)w.size();
                    w[ha + 1] = (uint32_t)per[ob].size();
                    w.insert(w.end(), per[ob].begin(), per[ob].end());
                }
            }
            if (p.nB < 0) {
                for (auto &w : bp) w[hb + 1] = kAll;
            } else {
                std::vector<std::vector<uint32_t>> per(g.n_blocks);
                for (int32_t v = 0; v < p.nB; ++v) {
                    const uint32_t e = lists[p.offB + v];
                    const int32_t s = (int32_t)(e & 0x7FFFu), d = (int32_t)((e >> 15) & 0x7FFFu);
                    const int32_t bk = blk_of[s];
                    if (blk_of[d] != bk)
                        return fail(FSV_EINVAL, "internal: beta pair leaves its block (operator %d)", i + jj);
                    const uint32_t c0 = (uint32_t)blocks[bk].x;
                    per[bk].push_back(((uint32_t)s - c0) | (((uint32_t)d - c0) << 15) | (e & 0x80000000u));
                }
                for (int32_t bk = 0; bk < g.n_blocks; ++bk) {
                    std::vector<uint32_t> &w = bp[bk];
                    w[hb] = (uint32_t)w.size();
                    w[hb + 1] = (uint32_t)per[bk].size();
                    w.insert(w.end(), per[bk].begin(), per[bk].end());
                }
            }
        }
        size_t as = 0, bs = 0;
        for (auto &w : ap) as = std::max(as, w.size());
        for (auto &w : bp) bs = std::max(bs, w.size());
        g.astride = (int32_t)((as + 3) & ~(size_t)3);
        g.bstride = (int32_t)((bs + 3) & ~(size_t)3);
        g.lds = 16 * (size_t)nops + (size_t)g.rmax * g.lmax * o.es * o.arrays +
                4 * ((size_t)g.astride + g.bstride + nops);
        if (g.lds > o.lds_limit) {  // programs too large for this run: one launch per operator
            for (int k = i; k < j; ++k) single(k);
            i = j;
            continue;
        }
        g.aprog_off = (int64_t)aprog.size();
        for (auto &w : ap) {
            w.resize(g.astride, 0u);
            aprog.insert(aprog.end(), w.begin(), w.end());
        }
        g.bprog_off = (int64_t)bprog.size();
        for (auto &w : bp) {
            w.resize(g.bstride, 0u);
            bprog.insert(bprog.end(), w.begin(), w.end());
        }
        for (int k = i; k < j; ++k) S.count[k] = g.n_orbits * g.n_blocks;
        S.groups.push_back(g);
        i = j;
    }
    // bounds of every tile program as k_fused reads it: rows of an orbit are
    // alpha ranks, a block is a column range of C, local pairs stay inside the
    // tile and each operator's list lies inside the program
    for (const FGroup &g : S.groups) {
        if (!g.fused) continue;
        if ((int64_t)g.n_orbits * g.n_blocks > o.max_tiles || g.rmax > kMaxTileRows || g.lmax > kMaxTileCols ||
            g.lds > o.lds_limit)
            return fail(FSV_EINVAL, "internal: tile run at operator %d exceeds its limits", g.k0);
        for (int32_t ob = 0; ob < g.n_orbits; ++ob) {
            const uint32_t *w = &aprog[(size_t)g.aprog_off + (size_t)ob * g.astride];
            const uint32_t nr = w[0];
            if (nr < 1 || nr > (uint32_t)g.rmax) return fail(FSV_EINVAL, "internal: tile orbit size");
            for (uint32_t t = 0; t < nr; ++t)
                if ((int64_t)w[1 + t] >= nsa) return fail(FSV_EINVAL, "internal: tile row rank");
            for (int jj = 0; jj < g.nops; ++jj) {
                const uint32_t off = w[1 + g.rmax + 2 * jj], cnt = w[2 + g.rmax + 2 * jj];
                if (cnt == kAll) continue;
                if ((size_t)off + cnt > (size_t)g.astride) return fail(FSV_EINVAL, "internal: tile alpha list");
                for (uint32_t u = 0; u < cnt; ++u) {
                    const uint32_t e = w[off + u];
                    if ((e & 0xFFu) >= nr || ((e >> 8) & 0xFFu) >= nr) return fail(FSV_EINVAL, "internal: tile alpha pair");
                }
            }
        }
        for (int32_t bk = 0; bk < g.n_blocks; ++bk) {
            const uint32_t *w = &bprog[(size_t)g.bprog_off + (size_t)bk * g.bstride];
            const uint32_t c0 = w[0], L = w[1];
            if (L < 1 || L > (uint32_t)g.lmax || (int64_t)c0 + L > nsb) return fail(FSV_EINVAL, "internal: tile block");
            for (int jj = 0; jj < g.nops; ++jj) {
                const uint32_t off = w[2 + 2 * jj], cnt = w[3 + 2 * jj];
                if (cnt == kAll) continue;
                if ((size_t)off + cnt > (size_t)g.bstride) return fail(FSV_EINVAL, "internal: tile beta list");
                for (uint32_t v = 0; v < cnt; ++v) {
                    const uint32_t e = w[off + v];
                    if ((e & 0x7FFFu) >= L || ((e >> 15) & 0x7FFFu) >= L) return fail(FSV_EINVAL, "internal: tile beta pair");
                }
            }
        }
    }
    auto up = [&](const std::vector<uint32_t> &vec, uint32_t **dst) -> int {
        void *p = nullptr;
        const size_t bytes = std::max<size_t>(vec.size(), 1) * 4;
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            return fail(FSV_ENOMEM, "hipMalloc of %zu bytes for fused programs failed", bytes);
        }
        S.mem.emplace_back(p, [](void *q) { (void)hipFree(q); });
        S.bytes += bytes;
        if (!vec.empty() && hipMemcpy(p, vec.data(), vec.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
            return fail(FSV_EDEVICE, "upload of fused programs failed");
        *dst = (uint32_t *)p;
        return FSV_OK;
    };
    int rc;
    if ((rc = up(aprog, &S.d_aprog)) || (rc = up(bprog, &S.d_bprog))) {
        S.release();
        return rc;
    }
    return FSV_OK;
}

int fused_runs(const FusedSched &S, int *n_fused_ops) {
    int runs = 0, nops = 0;
    for (const FGroup &g : S.groups)
        if (g.fused) {
            ++runs;
            nops += g.nops;
        }
    if (n_fused_ops) *n_fused_ops = nops;
    return runs;
}

void init_fused_kernels() {
    static bool done = false;
    if (done) return;
    done = true;
    const void *fns[] = {(const void *)k_fused<double, false>, (const void *)k_fused<double, true>,
                         (const void *)k_fused<float, false>, (const void *)k_fused<float, true>};
    for (const void *f : fns) {
        hipFuncAttributes fa;
        size_t lim = 163840;
        if (hipFuncGetAttributes(&fa, f) == hipSuccess) lim -= fa.sharedSizeBytes;
        (void)hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lim);
    }
    (void)hipGetLastError();
}

// Dynamic LDS every fused kernel accepts (their static LDS is the block_sum
// scratch of the adjoint kernels).
size_t fused_lds_limit() {
    init_fused_kernels();
    size_t lim = 163840;
    hipFuncAttributes fa;
    if (hipFuncGetAttributes(&fa, (const void *)k_fused<double, true>) == hipSuccess &&
        fa.maxDynamicSharedSizeBytes > 0)
        lim = std::min(lim, (size_t)fa.maxDynamicSharedSizeBytes);
    else
        lim = 65536 - 256;
    (void)hipGetLastError();
    return lim;
}

hipError_t launch_fused(int vtype, bool adjoint, void *psi, void *lam, const FusedSched &S, const FGroup &g,
                        const PairOp *d_pops, const double *cs, int64_t nsb, double *gpart, int gstride,
                        hipStream_t st) {
    if (g.fused == 2) return hipErrorInvalidValue;
    FArgs a;
    a.k0 = g.k0;
    a.nops = g.nops;
    a.n_blocks = g.n_blocks;
    a.gstride = gstride;
    a.astride = g.astride;
    a.bstride = g.bstride;
    a.rmax = g.rmax;
    a.lmax = g.lmax;
    a.nsb = nsb;
    a.aprog = S.d_aprog + g.aprog_off;
    a.bprog = S.d_bprog + g.bprog_off;
    a.ops = d_pops;
    a.cs = cs;
    const dim3 grid((unsigned)((int64_t)g.n_orbits * g.n_blocks)), block(kFusedBlock);
    if (vtype == V_F64) {
        if (adjoint)
            hipLaunchKernelGGL((k_fused<double, true>), grid, block, g.lds, st, (double *)psi, (double *)lam, a, gpart);
        else
            hipLaunchKernelGGL((k_fused<double, false>), grid, block, g.lds, st, (double *)psi, (double *)lam, a, gpart);
    } else if (vtype == V_F32) {
        if (adjoint)
            hipLaunchKernelGGL((k_fused<float, true>), grid, block, g.lds, st, (float *)psi, (float *)lam, a, gpart);
        else
            hipLaunchKernelGGL((k_fused<float, false>), grid, block, g.lds, st, (float *)psi, (float *)lam, a, gpart);
    } else {
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace fsv
