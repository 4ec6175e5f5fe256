// Fused runs of excitation rotations on the sector state, by connected
// components ("packets").
//
// The rotation of one operator mixes the two amplitudes of each of its active
// pairs and leaves every other amplitude alone.  For a run of consecutive
// operators, join two amplitudes whenever some operator of the run pairs them:
// the connected components of that graph are independent of each other, so
// each can be carried through the whole run on its own.  For the 24-qubit
// workloads (853,776 sector amplitudes, random singles and doubles) runs of
// about a dozen operators still have every component at or below 256
// amplitudes, while a single operator moves only ~15% of the state: a run
// becomes one launch over the ~85% of the state it touches instead of a dozen
// latency-bound launches.
//
// The host computes the components (union-find with union by size and
// rollback, so that a run is extended operator by operator while its largest
// component fits) and packs whole components into packets of at most 256
// amplitudes, row group by row group (rows that some component joins).  Per packet it stores the
// global indices of its amplitudes (ascending) and a region holding a header
// (amplitude count, then the cumulative pair count after each operator) and,
// operator by operator, the packet-local pairs as 16-bit words (first slot |
// second slot << 8).  The pair's sign is carried by the order of the slots:
// swapping the two amplitudes of a pair turns a rotation by -theta into one
// by +theta, and negates its gradient term, so every stored pair is applied
// with the positive sign.  One wavefront
// per packet: it loads the indices and the region in one round, gathers the
// amplitudes into LDS (lane l holds slots l, l + 64, l + 128, l + 192, so
// each load instruction covers 64 consecutive sorted indices), applies the run there (forward:
// rotations in order; adjoint: for the last operator back to the first, the
// gradient contribution, then psi and lam un-rotated) and scatters them back.
// The adjoint sweep keeps psi and lam of each amplitude side by side in
// memory, so a gather or scatter moves both in one access.  Untouched
// amplitudes are never read.  Consecutive workgroup ids go to
// different XCDs, so packet numbers are remapped to give each XCD a contiguous
// range of packets: with packets laid out by row group, the packets that
// share a cache line then share that XCD's L2.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <memory>
#include <vector>

#include "fsv_device.h"
#include "fsv_internal.h"

namespace fsv {

namespace {

constexpr int kPkt = kPacketAmps;    // amplitudes per packet (4 per lane)
constexpr int kPktHdr = 32;          // header words of a region
constexpr int kPktMaxOps = 15;       // operators per run: 15 x 128 16-bit pairs + header <= kPktMaxWords
constexpr int kPktMaxWords = 1024;   // region words (header + pairs)
constexpr uint32_t kNone = 0xFFFFFFFFu;  // padding of the index list
// an operator's pairs in one packet are disjoint: at most kPkt / 2 of them
static_assert(kPktHdr + kPktMaxOps * (kPkt / 2) / 2 <= kPktMaxWords, "packet region bound");
static_assert(kPktMaxOps <= 16, "gradient sums take 16 values per lane");
constexpr int kPktScalars = 2 * 16;  // LDS doubles: angles of <= 16 operators

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct PArgs {
    int32_t k0, m, wr, n_packets, gstride;
    const double *cs;
    int32_t store;  // 0: the run's results are not needed (the adjoint sweep's last run)
};

// Packet of workgroup slot v: XCD v % 8 gets a contiguous range of packets.
__device__ __forceinline__ int xcd_packet(int v, int n) {
    const int per = n >> 3, rem = n & 7, x = v & 7, i = v >> 3;
    return x * per + min(x, rem) + i;
}

// psi and lam of one slot side by side in LDS (one 16- or 8-byte access)
template <typename T> struct Slot2;
template <> struct Slot2<double> {
    using V = double2;
    static __device__ __forceinline__ V make(double a, double b) { return make_double2(a, b); }
};
template <> struct Slot2<float> {
    using V = float2;
    static __device__ __forceinline__ V make(float a, float b) { return make_float2(a, b); }
};

// One DPP lane move of a double (two 32-bit moves); lanes of rows outside RM
// receive 0.
template <int CTRL, int RM>
__device__ __forceinline__ double dpp_move(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, RM, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, RM, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sums over the 64 lanes of 16 values at once (a transposing butterfly):
// at each exchange a lane keeps half of its values and sends the other half
// to its partner, which keeps the opposite half, so 8 + 4 + 2 + 1 exchanges
// (then two of one value) replace 16 separate six-step sums.  Lanes differing
// in bit 0 and bit 1 exchange through DPP quad permutations, the others
// through lane shuffles.  On return lane l holds the total of value
// 8 b0 + 4 b1 + 2 b2 + b3 (b = the low bits of l); every row of 16 lanes holds
// all 16 totals.
__device__ __forceinline__ double wave_sum16(const double (&v)[16]) {
    const int l = threadIdx.x & (kWave - 1);
    const bool b0 = l & 1, b1 = l & 2, b2 = l & 4, b3 = l & 8;
    double w8[8], w4[4], w2[2];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
        const double keep = b0 ? v[r + 8] : v[r], send = b0 ? v[r] : v[r + 8];
        w8[r] = keep + dpp_move<0xB1, 0xF>(send);  // quad_perm [1, 0, 3, 2]: lane ^ 1
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const double keep = b1 ? w8[r + 4] : w8[r], send = b1 ? w8[r] : w8[r + 4];
        w4[r] = keep + dpp_move<0x4E, 0xF>(send);  // quad_perm [2, 3, 0, 1]: lane ^ 2
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
        const double keep = b2 ? w4[r + 2] : w4[r], send = b2 ? w4[r] : w4[r + 2];
        w2[r] = keep + __shfl_xor(send, 4, kWave);
    }
    double w = (b3 ? w2[1] : w2[0]) + __shfl_xor(b3 ? w2[0] : w2[1], 8, kWave);
    w += __shfl_xor(w, 16, kWave);
    w += __shfl_xor(w, 32, kWave);
    return w;
}

// The value whose total lane l holds after wave_sum16.
__device__ __forceinline__ int wave_sum16_index(int l) {
    return ((l & 1) << 3) | ((l & 2) << 1) | ((l & 4) >> 1) | ((l & 8) >> 3);
}

template <typename T>
__device__ __forceinline__ void rotp(T &a, T &b, T c, T s) {
    const T t = a;
    a = c * a - s * b;
    b = c * b + s * t;
}

// Streaming (non-temporal) stores of the scatter: a launch's results are read
// by the next launch, mostly on other XCDs, so they need not stay in this
// XCD's L2 (measured: 0.7 us less per adjoint launch at 24 qubits).
template <typename T>
__device__ __forceinline__ void store_stream(T *p, T v) {
    __builtin_nontemporal_store(v, p);
}
template <typename V2>
__device__ __forceinline__ void store_stream2(V2 *p, V2 v) {
    typedef decltype(v.x) E;
    typedef E E2 __attribute__((ext_vector_type(2)));
    E2 u;
    u.x = v.x;
    u.y = v.y;
    __builtin_nontemporal_store(u, (E2 *)p);
}
__device__ __forceinline__ void store_stream(double2 *p, double2 v) { store_stream2(p, v); }
__device__ __forceinline__ void store_stream(float2 *p, float2 v) { store_stream2(p, v); }

// Forward: psi is the state.  Adjoint: z holds (psi, lam) of each amplitude
// side by side, so one 16-byte (FP32: 8-byte) access moves both.
template <typename T, bool ADJ, int NQ>
__global__ __launch_bounds__(kWave) void k_pkt(T *__restrict__ psi, typename Slot2<T>::V *__restrict__ z,
                                               const uint32_t *__restrict__ ent,
                                               const uint32_t *__restrict__ reg, PArgs a,
                                               double *__restrict__ gpart) {
    extern __shared__ double lds[];
    double *scs = lds;  // cos, sin of the run's operators
    using V2 = typename Slot2<T>::V;
    T *tp = (T *)(lds + kPktScalars);  // forward: psi by slot
    V2 *tv = (V2 *)tp;                 // adjoint: (psi, lam) by slot
    uint32_t *rg = (uint32_t *)(tp + (ADJ ? 2 : 1) * kPkt);
    const int l = threadIdx.x;
    {
        const int t = min(l, 2 * a.m - 1);
        const double v = a.cs[2 * a.k0 + t];
        if (l < 2 * a.m) scs[l] = v;
    }
    double acc[16];  // this lane's share of each operator's gradient term (sweep order; 16th unused)
#pragma unroll
    for (int jj = 0; jj < 16; ++jj) acc[jj] = 0.0;
    const int nq = a.wr >> 2;
    for (int v = blockIdx.x; v < a.n_packets; v += gridDim.x) {
        const int p = xcd_packet(v, a.n_packets);
        // one round: indices and region (clamped, so every load is in flight at once)
        const uint32_t *es = ent + (size_t)p * kPkt;
        const u32x4 *rs = (const u32x4 *)(reg + (size_t)p * a.wr);
        uint32_t x[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) x[i] = es[l + i * kWave];  // slot l + 64 i
        u32x4 q[NQ];
#pragma unroll
        for (int i = 0; i < NQ; ++i) q[i] = rs[min(l + i * kWave, nq - 1)];
        T v0[4], v1[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t xi = x[i] == kNone ? 0u : x[i];
            if (ADJ) {
                const V2 zi = z[xi];
                v0[i] = zi.x;
                v1[i] = zi.y;
            } else {
                v0[i] = psi[xi];
            }
        }
        __syncthreads();  // the previous packet is out of LDS
        // Unconditional LDS writes: a clamped lane writes the value its
        // neighbour writes, and padding slots are never named by a pair.
#pragma unroll
        for (int i = 0; i < NQ; ++i) ((u32x4 *)rg)[min(l + i * kWave, nq - 1)] = q[i];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (ADJ)
                tv[l + i * kWave] = Slot2<T>::make(v0[i], v1[i]);
            else
                tp[l + i * kWave] = v0[i];
        }
        __syncthreads();
        // Operator jj of the sweep order (adjoint: last to first).  Its pair
        // range and each lane's first pair word are read before the loop, so
        // a step waits only for its amplitudes; gradient contributions stay
        // per lane in registers and are reduced once, after the packets.
        const uint32_t *rp = rg + kPktHdr;  // the pairs, two 16-bit words per 32-bit word
        const uint32_t npmax = 2u * (uint32_t)(a.wr - kPktHdr) - 1u;
        auto pair_at = [&](uint32_t t) { return (rp[t >> 1] >> ((t & 1u) << 4)) & 0xFFFFu; };
        uint32_t ob[kPktMaxOps], oe[kPktMaxOps], w0[kPktMaxOps];
#pragma unroll
        for (int jj = 0; jj < kPktMaxOps; ++jj) {
            const int j = ADJ ? a.m - 1 - jj : jj;
            const int jc = max(j, 0);
            ob[jj] = jc ? rg[jc] : 0u;
            oe[jj] = rg[1 + jc];
        }
#pragma unroll
        for (int jj = 0; jj < kPktMaxOps; ++jj) w0[jj] = pair_at(min(ob[jj] + l, npmax));
#pragma unroll
        for (int jj = 0; jj < kPktMaxOps; ++jj) {
            if (jj < a.m) {
                const int j = ADJ ? a.m - 1 - jj : jj;
                const T c = (T)scs[2 * j], s = (T)scs[2 * j + 1];
                uint32_t w = w0[jj];
                for (uint32_t t = ob[jj] + l; t < oe[jj]; t += kWave) {
                    if (t != ob[jj] + l) w = pair_at(t);
                    const int xs = (int)(w & 0xFFu), xd = (int)(w >> 8);
                    if (ADJ) {
                        const V2 A = tv[xs], B = tv[xd];
                        T va = A.x, la = A.y, vb = B.x, lb = B.y;
                        acc[jj] += (double)lb * (double)va - (double)la * (double)vb;
                        rotp(va, vb, c, -s);  // U^+ = U(-theta)
                        rotp(la, lb, c, -s);
                        tv[xs] = Slot2<T>::make(va, la);
                        tv[xd] = Slot2<T>::make(vb, lb);
                    } else {
                        T va = tp[xs], vb = tp[xd];
                        rotp(va, vb, c, s);
                        tp[xs] = va;
                        tp[xd] = vb;
                    }
                }
                __syncthreads();
            }
        }
        if (a.store) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (x[i] != kNone) {
                    if (ADJ)
                        store_stream(&z[x[i]], tv[l + i * kWave]);
                    else
                        store_stream(&psi[x[i]], tp[l + i * kWave]);
                }
        }
    }
    if (ADJ) {
        const double t = wave_sum16(acc);
        const int jj = wave_sum16_index(l);
        if (l < 16 && jj < a.m) gpart[(size_t)(a.k0 + a.m - 1 - jj) * a.gstride + blockIdx.x] = t;
    }
}

// Batched form: one launch carries one run of many independent instances.
// Each packet's header also holds (word kBHdr + ...) its instance's first
// amplitude in the arena (two words), the instance dimension (lam follows
// psi), the global index of the run's first operator (angles, gradients), the
// run length and the packet's gradient slot within its run; the gradient
// terms of each packet go to gpart[op * pstride + slot].
constexpr int kBHdr = 16;
static_assert(kBHdr > kPktMaxOps, "batched header fields follow the pair offsets");

template <bool ADJ, int NQ>
__global__ __launch_bounds__(kWave) void k_bpkt(double *__restrict__ arena, const uint32_t *__restrict__ ent,
                                                const uint32_t *__restrict__ reg, int wr, int n_packets,
                                                const double *__restrict__ cs, double *__restrict__ gpart,
                                                int pstride) {
    extern __shared__ double lds[];
    double *scs = lds;
    double *tp = lds + kPktScalars;  // forward: psi by slot
    double2 *tv = (double2 *)tp;     // adjoint: (psi, lam) by slot
    uint32_t *rg = (uint32_t *)(tp + (ADJ ? 2 : 1) * kPkt);
    const int l = threadIdx.x;
    const int nq = wr >> 2;
    for (int v = blockIdx.x; v < n_packets; v += gridDim.x) {
        const int p = xcd_packet(v, n_packets);
        const uint32_t *es = ent + (size_t)p * kPkt;
        const u32x4 *rs = (const u32x4 *)(reg + (size_t)p * wr);
        uint32_t x[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) x[i] = es[l + i * kWave];
        u32x4 q[NQ];
#pragma unroll
        for (int i = 0; i < NQ; ++i) q[i] = rs[min(l + i * kWave, nq - 1)];
        __syncthreads();  // the previous packet is out of LDS
#pragma unroll
        for (int i = 0; i < NQ; ++i) ((u32x4 *)rg)[min(l + i * kWave, nq - 1)] = q[i];
        __syncthreads();
        const int64_t base = (int64_t)rg[kBHdr] | ((int64_t)rg[kBHdr + 1] << 32);
        const int64_t dim = rg[kBHdr + 2];
        // the same for every lane: keep them scalar
        const int k0 = __builtin_amdgcn_readfirstlane((int)rg[kBHdr + 3]);
        const int m = __builtin_amdgcn_readfirstlane((int)rg[kBHdr + 4]);
        const int slot = __builtin_amdgcn_readfirstlane((int)rg[kBHdr + 5]);
        double *psi = arena + base, *lam = psi + dim;
        {
            const int t = min(l, max(2 * m - 1, 0));
            const double c = cs[2 * k0 + t];
            if (l < 2 * m) scs[l] = c;
        }
        double v0[4], v1[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const uint32_t xi = x[i] == kNone ? 0u : x[i];
            v0[i] = psi[xi];
            if (ADJ) v1[i] = lam[xi];
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (ADJ)
                tv[l + i * kWave] = make_double2(v0[i], v1[i]);
            else
                tp[l + i * kWave] = v0[i];
        }
        __syncthreads();
        const uint32_t *rp = rg + kPktHdr;
        auto pair_at = [&](uint32_t t) { return (rp[t >> 1] >> ((t & 1u) << 4)) & 0xFFFFu; };
        double acc[16];
        acc[15] = 0.0;
#pragma unroll
        for (int jj = 0; jj < kPktMaxOps; ++jj) {
            acc[jj] = 0.0;
            if (jj < m) {
                const int j = ADJ ? m - 1 - jj : jj;
                const uint32_t o0 = j ? rg[j] : 0u, o1 = rg[1 + j];
                const double c = scs[2 * j], sn = scs[2 * j + 1];
                for (uint32_t t = o0 + l; t < o1; t += kWave) {
                    const uint32_t w = pair_at(t);
                    const int xs = (int)(w & 0xFFu), xd = (int)(w >> 8);
                    if (ADJ) {
                        const double2 A = tv[xs], B = tv[xd];
                        double va = A.x, la = A.y, vb = B.x, lb = B.y;
                        acc[jj] += lb * va - la * vb;
                        rotp(va, vb, c, -sn);
                        rotp(la, lb, c, -sn);
                        tv[xs] = make_double2(va, la);
                        tv[xd] = make_double2(vb, lb);
                    } else {
                        double va = tp[xs], vb = tp[xd];
                        rotp(va, vb, c, sn);
                        tp[xs] = va;
                        tp[xd] = vb;
                    }
                }
                __syncthreads();
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (x[i] != kNone) {
                if (ADJ) {
                    const double2 A = tv[l + i * kWave];
                    psi[x[i]] = A.x;
                    lam[x[i]] = A.y;
                } else {
                    psi[x[i]] = tp[l + i * kWave];
                }
            }
        if (ADJ) {
            const double t = wave_sum16(acc);
            const int jj = wave_sum16_index(l);
            if (l < 16 && jj < m) gpart[(size_t)(k0 + m - 1 - jj) * pstride + slot] = t;
        }
    }
}

// ---- host: union-find over the amplitudes touched by a run ----
struct UnionFind {
    std::vector<int32_t> parent, size, comp;
    std::vector<uint8_t> seen;
    std::vector<int32_t> touched, log;
    explicit UnionFind(int64_t n) : parent(n), size(n, 1), comp(n, -1), seen(n, 0) {
        for (int64_t i = 0; i < n; ++i) parent[i] = (int32_t)i;
    }
    int32_t find(int32_t x) const {  // union by size keeps the depth <= log2(kPkt)
        while (parent[x] != x) x = parent[x];
        return x;
    }
    void mark(int32_t x) {
        if (!seen[x]) {
            seen[x] = 1;
            touched.push_back(x);
        }
    }
    int32_t unite(int32_t x, int32_t y) {  // size of the joined component
        int32_t rx = find(x), ry = find(y);
        if (rx == ry) return size[rx];
        if (size[rx] < size[ry]) std::swap(rx, ry);
        parent[ry] = rx;
        size[rx] += size[ry];
        log.push_back(ry);
        return size[rx];
    }
    void rollback(size_t lmark, size_t tmark) {
        for (size_t t = log.size(); t-- > lmark;) {
            const int32_t ry = log[t], rx = parent[ry];
            size[rx] -= size[ry];
            parent[ry] = ry;
        }
        log.resize(lmark);
        for (size_t t = tmark; t < touched.size(); ++t) seen[touched[t]] = 0;
        touched.resize(tmark);
    }
    void reset() {
        for (int32_t x : touched) {
            parent[x] = x;
            size[x] = 1;
            comp[x] = -1;
            seen[x] = 0;
        }
        touched.clear();
        log.clear();
    }
};

// Calls f(src, dst, neg) for every active pair of operator op; stops early
// when f returns false.
template <typename F>
bool for_pairs(const PairOp &op, const std::vector<uint32_t> &lists, int64_t nsa, int64_t nsb, F &&f) {
    const int64_t na = op.nA >= 0 ? op.nA : nsa, nb = op.nB >= 0 ? op.nB : nsb;
    for (int64_t u = 0; u < na; ++u) {
        int64_t ia = u, ia2 = u;
        bool nrow = op.sign0 < 0;
        if (op.nA >= 0) {
            const uint32_t e = lists[op.offA + u];
            ia = e & 0x7FFFu;
            ia2 = (e >> 15) & 0x7FFFu;
            nrow ^= (e >> 31) != 0;
        }
        for (int64_t v = 0; v < nb; ++v) {
            int64_t ib = v, ib2 = v;
            bool neg = nrow;
            if (op.nB >= 0) {
                const uint32_t e = lists[op.offB + v];
                ib = e & 0x7FFFu;
                ib2 = (e >> 15) & 0x7FFFu;
                neg ^= (e >> 31) != 0;
            }
            if (!f((int32_t)(ia * nsb + ib), (int32_t)(ia2 * nsb + ib2), neg)) return false;
        }
    }
    return true;
}

int upload_words(const std::vector<uint32_t> &vec, FusedSched &S, uint32_t **dst) {
    void *p = nullptr;
    const size_t bytes = std::max<size_t>(vec.size(), 1) * 4;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return fail(FSV_ENOMEM, "hipMalloc of %zu bytes for packet programs failed", bytes);
    }
    S.mem.emplace_back(p, [](void *q) { (void)hipFree(q); });
    S.bytes += bytes;
    if (!vec.empty() && hipMemcpy(p, vec.data(), vec.size() * 4, hipMemcpyHostToDevice) != hipSuccess)
        return fail(FSV_EDEVICE, "upload of packet programs failed");
    *dst = (uint32_t *)p;
    return FSV_OK;
}

// Packing of whole components into packets of at most kPkt amplitudes.  A
// packet is started with the first unpacked component in `order` (row group
// by row group), then grown greedily with the component that shares the most
// 128-byte lines of the 8-byte state (16 amplitudes) with what the packet
// already holds (ties: earlier in `order`), or, when no such component fits,
// with the earliest unpacked one in `order` that fits (a queue per size).
// Every component touching a line lies in the line's row group, so packets
// still follow the group order.  pk_of[c] = packet of component c; returns
// the packet count.
struct PackScratch {
    std::vector<int32_t> cstart, cmem, lstart, lcomp, pos, score, cand, plines, cnt;
    std::vector<uint8_t> done, lin;
    std::vector<std::vector<int32_t>> bysize;  // unpacked components of each size, in order
    std::vector<size_t> head;
};

int pack_by_lines(const std::vector<int32_t> &tv, UnionFind &uf, const std::vector<int32_t> &csize,
                  const std::vector<int32_t> &order, std::vector<int32_t> &pk_of, PackScratch &w,
                  const std::vector<uint8_t> *skip = nullptr) {
    const int nc = (int)csize.size();
    const int no = (int)order.size();  // the components to pack (all, or those not skipped)
    constexpr int kLineShift = 4;
    pk_of.assign(nc, -1);
    if (nc == 0) return 0;
    // lines of each component (ascending, distinct): tv is sorted, so a
    // component's members arrive in ascending order
    w.cstart.assign(nc + 1, 0);
    for (int32_t x : tv) ++w.cstart[uf.comp[uf.find(x)] + 1];
    for (int c = 0; c < nc; ++c) w.cstart[c + 1] += w.cstart[c];
    w.cmem.assign(tv.size(), 0);
    w.cnt.assign(w.cstart.begin(), w.cstart.end() - 1);
    for (int32_t x : tv) {
        const int c = uf.comp[uf.find(x)];
        const int32_t ln = x >> kLineShift;
        const int at = w.cnt[c];
        if (at == w.cstart[c] || w.cmem[at - 1] != ln) w.cmem[w.cnt[c]++] = ln;
    }
    // line -> components (CSR over the lines that occur)
    const int32_t nl = (tv.back() >> kLineShift) + 1;
    w.lstart.assign((size_t)nl + 1, 0);
    for (int c = 0; c < nc; ++c)
        for (int t = w.cstart[c]; t < w.cnt[c]; ++t) ++w.lstart[w.cmem[t] + 1];
    for (int32_t l = 0; l < nl; ++l) w.lstart[l + 1] += w.lstart[l];
    w.lcomp.assign(w.lstart[nl], 0);
    std::vector<int32_t> &lfill = w.plines;  // reused as a cursor per line
    lfill.assign(w.lstart.begin(), w.lstart.end() - 1);
    for (int c = 0; c < nc; ++c)
        for (int t = w.cstart[c]; t < w.cnt[c]; ++t) w.lcomp[lfill[w.cmem[t]]++] = c;
    w.pos.assign(nc, 0);
    for (int t = 0; t < no; ++t) w.pos[order[t]] = t;
    w.done.assign(nc, 0);
    if (skip)
        for (int c = 0; c < nc; ++c) w.done[c] = (*skip)[c];
    w.score.assign(nc, 0);
    w.lin.assign((size_t)nl, 0);
    w.plines.clear();
    w.bysize.assign(kPkt + 1, {});
    w.head.assign(kPkt + 1, 0);
    for (int t = 0; t < no; ++t) w.bysize[csize[order[t]]].push_back(order[t]);
    int npk = 0;
    size_t si = 0;
    while (true) {
        while (si < (size_t)no && w.done[order[si]]) ++si;
        if (si == (size_t)no) break;
        const int p = npk++;
        int fill = 0;
        w.cand.clear();
        auto add = [&](int c) {
            w.done[c] = 1;
            pk_of[c] = p;
            fill += csize[c];
            for (int t = w.cstart[c]; t < w.cnt[c]; ++t) {
                const int32_t ln = w.cmem[t];
                if (w.lin[ln]) continue;
                w.lin[ln] = 1;
                w.plines.push_back(ln);
                for (int32_t u = w.lstart[ln]; u < w.lstart[ln + 1]; ++u) {
                    const int d = w.lcomp[u];
                    if (!w.done[d] && w.score[d]++ == 0) w.cand.push_back(d);
                }
            }
        };
        add(order[si]);
        while (fill < kPkt) {
            int best = -1;
            for (int d : w.cand)
                if (!w.done[d] && fill + csize[d] <= kPkt &&
                    (best < 0 || w.score[d] > w.score[best] || (w.score[d] == w.score[best] && w.pos[d] < w.pos[best])))
                    best = d;
            if (best < 0)  // the earliest unpacked component (in order) that fits
                for (int sz = 1; sz <= kPkt - fill; ++sz) {
                    std::vector<int32_t> &q = w.bysize[sz];
                    size_t &h = w.head[sz];
                    while (h < q.size() && w.done[q[h]]) ++h;
                    if (h < q.size() && (best < 0 || w.pos[q[h]] < w.pos[best])) best = q[h];
                }
            if (best < 0) break;
            add(best);
        }
        for (int d : w.cand) w.score[d] = 0;
        for (int32_t ln : w.plines) w.lin[ln] = 0;
        w.plines.clear();
    }
    return npk;
}

// XCD placement of a run's components.  The workgroups of a launch are dealt
// to the 8 XCDs round robin, the kernel gives XCD x a contiguous range of
// packets, and each XCD has its own L2: a line that packets on several XCDs
// gather is fetched, and written back, once per XCD.  Starting from the
// packing by lines (contiguous ranges of its packets per XCD), a few passes
// in `order` move each component to the XCD that already holds the most of
// its lines of 8 amplitudes (one 128-byte line of the adjoint sweep's
// (psi, lam) pairs), keeping every XCD within 2 % of an even share of the
// amplitudes.  Each XCD's components are then packed by lines on their own,
// and the XCDs' packet lists are padded with empty packets to one length n,
// so that XCD x runs packets [x n, (x + 1) n).  At 24 qubits this takes the
// mean number of XCDs per touched line from 1.59 to 1.38.
int pack_by_xcd(const std::vector<int32_t> &tv, UnionFind &uf, const std::vector<int32_t> &csize,
                const std::vector<int32_t> &order, std::vector<int32_t> &pk_of, PackScratch &w) {
    constexpr int X = 8;
    const int nc = (int)csize.size();
    const int npk0 = pack_by_lines(tv, uf, csize, order, pk_of, w);
    // small runs, and runs of states far beyond the caches (whose placement
    // passes would cost seconds per run): the packing by lines as it is
    if (npk0 < 8 * X || npk0 > 16384) return npk0;
    std::vector<int8_t> part(nc);
    {
        const int per = npk0 / X, rem = npk0 % X;
        for (int c = 0; c < nc; ++c) {
            int x = 0;  // the XCD whose range [x per + min(x, rem), ...) holds the packet
            while (x + 1 < X && pk_of[c] >= (x + 1) * per + std::min(x + 1, rem)) ++x;
            part[c] = (int8_t)x;
        }
    }
    // lines of each component (ascending, distinct; tv is sorted)
    const size_t n = tv.size();
    std::vector<int32_t> lid(n), cof(n), cstart(nc + 1, 0), cl(n), cnt_c(nc, 0);
    int32_t nl = 0;
    for (size_t t = 0; t < n; ++t) {
        if (t == 0 || (tv[t] >> 3) != (tv[t - 1] >> 3)) ++nl;
        lid[t] = nl - 1;
        cof[t] = uf.comp[uf.find(tv[t])];
        ++cstart[cof[t] + 1];
    }
    for (int c = 0; c < nc; ++c) cstart[c + 1] += cstart[c];
    for (size_t t = 0; t < n; ++t) {
        const int c = cof[t];
        const int at = cstart[c] + cnt_c[c];
        if (cnt_c[c] == 0 || cl[at - 1] != lid[t]) {
            cl[at] = lid[t];
            ++cnt_c[c];
        }
    }
    std::vector<int32_t> cnt((size_t)nl * X, 0);
    int64_t load[X] = {0}, total = 0;
    for (int c = 0; c < nc; ++c) {
        for (int u = 0; u < cnt_c[c]; ++u) ++cnt[(size_t)cl[cstart[c] + u] * X + part[c]];
        load[part[c]] += csize[c];
        total += csize[c];
    }
    const int64_t cap = total * 102 / (100 * X) + 1;
    for (int pass = 0; pass < 3; ++pass) {
        int moved = 0;
        for (int t = 0; t < nc; ++t) {
            const int c = order[t], p0 = part[c];
            int pres[X] = {0};
            for (int u = 0; u < cnt_c[c]; ++u) {
                int32_t *row = &cnt[(size_t)cl[cstart[c] + u] * X];
                --row[p0];
                for (int q = 0; q < X; ++q) pres[q] += row[q] > 0;
            }
            int best = p0;
            for (int q = 0; q < X; ++q)
                if (q != p0 && load[q] + csize[c] <= cap && pres[q] > pres[best]) best = q;
            for (int u = 0; u < cnt_c[c]; ++u) ++cnt[(size_t)cl[cstart[c] + u] * X + best];
            if (best != p0) {
                load[p0] -= csize[c];
                load[best] += csize[c];
                part[c] = (int8_t)best;
                ++moved;
            }
        }
        if (!moved) break;
    }
    // pack each XCD's components by lines, then lay the XCDs out in equal ranges
    std::vector<uint8_t> skip(nc);
    std::vector<int32_t> ox, lk, local(nc, -1);
    int nmax = 0;
    for (int x = 0; x < X; ++x) {
        ox.clear();
        for (int t = 0; t < nc; ++t)
            if (part[order[t]] == x) ox.push_back(order[t]);
        for (int c = 0; c < nc; ++c) skip[c] = part[c] != x;
        const int nx = pack_by_lines(tv, uf, csize, ox, lk, w, &skip);
        for (int c : ox) local[c] = lk[c];
        nmax = std::max(nmax, nx);
    }
    for (int c = 0; c < nc; ++c) pk_of[c] = part[c] * nmax + local[c];
    return X * nmax;
}

}  // namespace

int64_t packet_max_dim() { return (int64_t)1 << 26; }
int64_t packet_default_dim() { return (int64_t)1 << 22; }

int plan_packets(int64_t nsa, int64_t nsb, const std::vector<PairOp> &pops, const std::vector<uint32_t> &lists,
                 const FusedOpts &o, bool every_run, PacketPlan &S) {
    S.groups.clear();
    S.ent.clear();
    S.reg.clear();
    const int K = (int)pops.size();
    S.count.assign(K, -1);
    const int64_t N = nsa * nsb;
    if (K == 0) return FSV_OK;
    if (N > packet_max_dim()) return fail(FSV_EINVAL, "internal: packet runs need at most %lld amplitudes",
                                          (long long)packet_max_dim());
    UnionFind uf(N);
    const bool verbose = std::getenv("FSV_VERBOSE") != nullptr;
    auto pairs_of = [&](const PairOp &p) {
        return (double)(p.nA >= 0 ? p.nA : nsa) * (double)(p.nB >= 0 ? p.nB : nsb);
    };
    // cost model (adjoint sweep, per-operator launches ~5 us each; a packet
    // run ~6 us of launch and load chain plus its bytes at ~2 TB/s)
    const double bw = 4.0e12, bw_pk = 2.0e12, t_launch = 5.0e-6, t_chain = 6.0e-6;
    const double amp = (double)o.es * 2;  // psi and lam
    const int max_ops = std::min(o.max_ops, kPktMaxOps);
    std::vector<uint32_t> &ent = S.ent, &reg = S.reg;
    std::vector<int32_t> csize, crow, order, pk_of, pfill, cnt, cur;
    PackScratch pk;
    std::vector<int32_t> slot(N, 0), pkt(N, 0), rpar(nsa);  // per touched amplitude: its slot and packet
    // support of the forward state from the reference (sector amplitude 0),
    // followed through the first runs while their nonzero packets are few
    bool track = !every_run;
    std::vector<uint8_t> nz, pmark, cmark;
    if (track) nz.assign(N, 0), nz[0] = 1;
    auto single = [&](int k) {
        FGroup s{};
        s.k0 = k;
        s.nops = 1;
        S.groups.push_back(s);
        track = false;  // one launch over all its pairs: the support is not followed further
    };
    int i = 0;
    while (i < K) {
        int j = i;
        while (j < K && j - i < max_ops) {
            const size_t lmark = uf.log.size(), tmark = uf.touched.size();
            const bool ok = for_pairs(pops[j], lists, nsa, nsb, [&](int32_t s, int32_t d, bool) {
                uf.mark(s);
                uf.mark(d);
                return uf.unite(s, d) <= kPkt;
            });
            if (!ok) {
                uf.rollback(lmark, tmark);
                break;
            }
            ++j;
        }
        const int m = j - i;
        bool fuse = m >= 2 && o.mode != 1 && !uf.touched.empty();
        double npairs = 0.0;
        for (int k = i; k < j; ++k) npairs += pairs_of(pops[k]);
        if (every_run) {
            fuse = true;  // every run becomes a packet run (one with no pairs has no packets)
        } else if (fuse && o.mode == 0) {
            const double t_ops = m * t_launch + npairs * 4.0 * amp / bw;
            const double t_pk = t_chain + ((double)uf.touched.size() * (2.0 * amp + 4.0) + npairs * 4.0) / bw_pk;
            fuse = t_pk < t_ops;
        }
        if (!fuse) {
            for (int k = i; k < j; ++k) single(k);
            uf.reset();
            i = j;
            continue;
        }
        // Components, numbered in order of their smallest amplitude.
        std::vector<int32_t> &tv = uf.touched;
        if ((int64_t)tv.size() * 8 > N) {  // most amplitudes touched: a scan of the marks beats a sort
            tv.clear();
            for (int64_t x = 0; x < N; ++x)
                if (uf.seen[x]) tv.push_back((int32_t)x);
        } else {
            std::sort(tv.begin(), tv.end());
        }
        // the run's unions are final: point every touched amplitude at its
        // root, so that the lookups below take one step (reset() undoes it)
        for (int32_t x : tv) uf.parent[x] = uf.find(x);
        csize.clear();
        crow.clear();
        for (int32_t x : tv) {
            const int32_t r = uf.find(x);
            if (uf.comp[r] < 0) {
                uf.comp[r] = (int32_t)csize.size();
                csize.push_back(uf.size[r]);
                crow.push_back((int32_t)(x / nsb));
            }
        }
        // Row groups: rows joined whenever one component has amplitudes in
        // both.  Every component touching a row lies in that row's group, so
        // a cache line (a segment of one row) is only ever touched by packets
        // of one group.  Packets are laid out group by group (groups in order
        // of their first row), and the kernel gives each XCD a contiguous
        // range of packets, so most lines live in one XCD's L2.
        for (int64_t r = 0; r < nsa; ++r) rpar[r] = (int32_t)r;
        auto rfind = [&](int32_t r) {
            while (rpar[r] != r) r = rpar[r] = rpar[rpar[r]];
            return r;
        };
        for (int32_t x : tv) {
            const int32_t a = rfind(crow[uf.comp[uf.find(x)]]), b = rfind((int32_t)(x / nsb));
            if (a != b) rpar[std::max(a, b)] = std::min(a, b);  // root = smallest row
        }
        order.resize(csize.size());
        for (size_t c = 0; c < order.size(); ++c) order[c] = (int32_t)c;
        std::stable_sort(order.begin(), order.end(),
                         [&](int32_t u, int32_t v) { return rfind(crow[u]) < rfind(crow[v]); });
        const int npk = o.place_xcd ? pack_by_xcd(tv, uf, csize, order, pk_of, pk)
                                    : pack_by_lines(tv, uf, csize, order, pk_of, pk);
        const size_t e0 = ent.size();
        ent.resize(e0 + (size_t)npk * kPkt, kNone);
        pfill.assign(npk, 0);
        for (int32_t x : tv) {
            const int pk = pk_of[uf.comp[uf.find(x)]];
            const int sl = pfill[pk]++;
            ent[e0 + (size_t)pk * kPkt + sl] = (uint32_t)x;
            slot[x] = sl;
            pkt[x] = pk;
        }
        // per packet and operator pair counts, then the regions
        cnt.assign((size_t)npk * m, 0);
        for (int jj = 0; jj < m; ++jj)
            for_pairs(pops[i + jj], lists, nsa, nsb, [&](int32_t s, int32_t, bool) {
                ++cnt[(size_t)pkt[s] * m + jj];
                return true;
            });
        int maxp = 0;
        for (int pk = 0; pk < npk; ++pk) {
            int t = 0;
            for (int jj = 0; jj < m; ++jj) t += cnt[(size_t)pk * m + jj];
            maxp = std::max(maxp, t);
        }
        const int wr = (kPktHdr + (maxp + 1) / 2 + 3) & ~3;
        if (wr > kPktMaxWords) return fail(FSV_EINVAL, "internal: packet region of %d words", wr);
        const size_t r0 = reg.size();
        reg.resize(r0 + (size_t)npk * wr, 0u);
        cur.assign((size_t)npk * m, 0);
        for (int pk = 0; pk < npk; ++pk) {
            uint32_t *h = &reg[r0 + (size_t)pk * wr];
            h[0] = (uint32_t)pfill[pk];
            int t = 0;
            for (int jj = 0; jj < m; ++jj) {
                cur[(size_t)pk * m + jj] = t;
                t += cnt[(size_t)pk * m + jj];
                h[1 + jj] = (uint32_t)t;
            }
        }
        for (int jj = 0; jj < m; ++jj)
            for_pairs(pops[i + jj], lists, nsa, nsb, [&](int32_t s, int32_t d, bool neg) {
                const int pk = pkt[s];
                const int at = cur[(size_t)pk * m + jj]++;
                const uint32_t v = neg ? (uint32_t)(slot[d] | (slot[s] << 8)) : (uint32_t)(slot[s] | (slot[d] << 8));
                reg[r0 + (size_t)pk * wr + kPktHdr + (at >> 1)] |= v << ((at & 1) << 4);
                return true;
            });
        FGroup g{};
        g.k0 = i;
        g.nops = m;
        g.fused = 2;
        g.n_packets = npk;
        g.wr = wr;
        g.ent_off = (int64_t)e0;
        g.reg_off = (int64_t)r0;
        if (track) {
            // packets holding a nonzero amplitude, and the components that
            // become nonzero (untouched amplitudes keep their values)
            pmark.assign(npk, 0);
            cmark.assign(csize.size(), 0);
            for (int32_t x : tv)
                if (nz[x]) {
                    const int c = uf.comp[uf.find(x)];
                    cmark[c] = 1;
                    pmark[pk_of[c]] = 1;
                }
            int nsel = 0;
            for (int q = 0; q < npk; ++q) nsel += pmark[q];
            if (2 * nsel > npk) {
                track = false;
            } else {
                for (int32_t x : tv)
                    if (cmark[uf.comp[uf.find(x)]]) nz[x] = 1;
                g.sub_n = nsel;
                g.sub_ent_off = (int64_t)ent.size();
                g.sub_reg_off = (int64_t)reg.size();
                ent.resize(ent.size() + (size_t)nsel * kPkt);
                reg.resize(reg.size() + (size_t)nsel * wr);
                for (int q = 0, t = 0; q < npk; ++q)
                    if (pmark[q]) {
                        std::copy_n(ent.begin() + e0 + (size_t)q * kPkt, kPkt,
                                    ent.begin() + g.sub_ent_off + (size_t)t * kPkt);
                        std::copy_n(reg.begin() + r0 + (size_t)q * wr, wr, reg.begin() + g.sub_reg_off + (size_t)t * wr);
                        ++t;
                    }
            }
        }
        if (verbose) {  // planning a large state takes minutes: one line per run
            std::fprintf(stderr, "[fsv] packet run at operator %d: %d operators, %d packets\n", i, m, npk);
            std::fflush(stderr);
        }
        g.lds = sizeof(double) * kPktScalars + (size_t)kPkt * 2 * o.es + (size_t)wr * 4;
        const int grid = std::min(npk, max_grid());
        for (int k = i; k < j; ++k) S.count[k] = grid;
        S.groups.push_back(g);
        uf.reset();
        i = j;
    }
    return FSV_OK;
}

// Bounds of one packet program (index list at ent[e0], region at reg[r0] of
// wr words) of a run of m operators, as the packet kernels read them: the
// index list holds h[0] ascending amplitude indices below dim (none in the
// empty packets that pad an XCD's range), then padding;
// the cumulative pair counts h[1..m] never decrease and fit the region; every
// pair names two distinct filled slots, and no slot appears in two pairs of
// one operator (the lanes of a wavefront apply an operator's pairs at once).
int check_packet(const std::vector<uint32_t> &ent, size_t e0, const std::vector<uint32_t> &reg, size_t r0, int wr,
                 int m, int64_t dim, const char *what) {
    if (e0 + kPkt > ent.size() || r0 + (size_t)wr > reg.size())
        return fail(FSV_EINVAL, "internal: %s program outside its table", what);
    const uint32_t *h = &reg[r0];
    const uint32_t fill = h[0];
    if (fill > (uint32_t)kPkt) return fail(FSV_EINVAL, "internal: %s holds %u amplitudes", what, fill);
    for (uint32_t t = 0; t < (uint32_t)kPkt; ++t) {
        const uint32_t x = ent[e0 + t];
        if (t < fill) {
            if ((int64_t)x >= dim || (t > 0 && x <= ent[e0 + t - 1]))
                return fail(FSV_EINVAL, "internal: %s index %u out of order or range", what, t);
        } else if (x != kNone) {
            return fail(FSV_EINVAL, "internal: %s padding slot %u is not empty", what, t);
        }
    }
    uint32_t prev = 0;
    std::vector<uint8_t> used(kPkt);
    for (int j = 0; j < m; ++j) {
        const uint32_t end = h[1 + j];
        if (end < prev || end > 2u * (uint32_t)(wr - kPktHdr))
            return fail(FSV_EINVAL, "internal: %s pair range of operator %d", what, j);
        std::fill(used.begin(), used.end(), 0);
        for (uint32_t t = prev; t < end; ++t) {
            const uint32_t w = (reg[r0 + kPktHdr + (t >> 1)] >> ((t & 1u) << 4)) & 0xFFFFu;
            const uint32_t a = w & 0xFFu, b = w >> 8;
            if (a >= fill || b >= fill || a == b || used[a] || used[b])
                return fail(FSV_EINVAL, "internal: %s pair %u of operator %d", what, t, j);
            used[a] = used[b] = 1;
        }
        prev = end;
    }
    return FSV_OK;
}

// Every program of every packet run (and of its forward-support copy).
int check_packet_plan(const PacketPlan &P, int64_t dim, int K) {
    for (const FGroup &g : P.groups) {
        if (g.k0 < 0 || g.nops < 1 || g.k0 + g.nops > K) return fail(FSV_EINVAL, "internal: run bounds");
        if (g.fused != 2) continue;
        if (g.nops > kPktMaxOps || g.wr < kPktHdr + 4 || g.wr > kPktMaxWords || (g.wr & 3) || g.n_packets < 0)
            return fail(FSV_EINVAL, "internal: packet run at operator %d has region %d", g.k0, g.wr);
        int rc;
        for (int q = 0; q < g.n_packets; ++q)
            if ((rc = check_packet(P.ent, (size_t)g.ent_off + (size_t)q * kPkt, P.reg, (size_t)g.reg_off + (size_t)q * g.wr,
                                   g.wr, g.nops, dim, "packet")))
                return rc;
        for (int q = 0; q < g.sub_n; ++q)
            if ((rc = check_packet(P.ent, (size_t)g.sub_ent_off + (size_t)q * kPkt, P.reg,
                                   (size_t)g.sub_reg_off + (size_t)q * g.wr, g.wr, g.nops, dim, "support packet")))
                return rc;
        if (g.sub_n > g.n_packets) return fail(FSV_EINVAL, "internal: support copy larger than its run");
        for (int k = g.k0; k < g.k0 + g.nops; ++k)
            if (P.count[k] != std::min(g.n_packets, max_grid()))
                return fail(FSV_EINVAL, "internal: gradient partial count of operator %d", k);
    }
    return FSV_OK;
}

int build_packets(int64_t nsa, int64_t nsb, const std::vector<PairOp> &pops, const std::vector<uint32_t> &lists,
                  const FusedOpts &o, FusedSched &S) {
    S.release();
    PacketPlan pp;
    int rc = plan_packets(nsa, nsb, pops, lists, o, false, pp);
    if (rc) return rc;
    if ((rc = check_packet_plan(pp, nsa * nsb, (int)pops.size()))) return rc;
    S.groups = std::move(pp.groups);
    S.count = std::move(pp.count);
    if ((rc = upload_words(pp.ent, S, &S.d_aprog)) || (rc = upload_words(pp.reg, S, &S.d_bprog))) {
        S.release();
        return rc;
    }
    S.packets = true;
    return FSV_OK;
}

namespace {

// t0 / t1 (optional): events that take the kernel's own start and end times.
template <typename T, bool ADJ>
hipError_t pkt_impl(void *state, const FusedSched &S, const FGroup &g, const double *cs, double *gpart, int gstride,
                    hipStream_t stream, hipEvent_t t0, hipEvent_t t1, bool store) {
    using V2 = typename Slot2<T>::V;
    PArgs a{g.k0, g.nops, g.wr, g.n_packets, gstride, cs, store ? 1 : 0};
    const uint32_t *ent = S.d_aprog + g.ent_off, *reg = S.d_bprog + g.reg_off;
    const uint32_t shm =
        (uint32_t)(sizeof(double) * kPktScalars + (size_t)kPkt * (ADJ ? 2 : 1) * sizeof(T) + (size_t)g.wr * 4);
    const dim3 grid((unsigned)std::min(g.n_packets, max_grid())), block(kWave);
    T *psi = ADJ ? nullptr : (T *)state;
    V2 *z = ADJ ? (V2 *)state : nullptr;
    const bool narrow = g.wr <= 4 * kWave * 2;  // else wr <= kPktMaxWords
    if (t0 || t1) {
        if (narrow)
            hipExtLaunchKernelGGL(k_pkt<T, ADJ, 2>, grid, block, shm, stream, t0, t1, 0u, psi, z, ent, reg, a, gpart);
        else
            hipExtLaunchKernelGGL(k_pkt<T, ADJ, 4>, grid, block, shm, stream, t0, t1, 0u, psi, z, ent, reg, a, gpart);
    } else if (narrow) {
        hipLaunchKernelGGL((k_pkt<T, ADJ, 2>), grid, block, shm, stream, psi, z, ent, reg, a, gpart);
    } else {
        hipLaunchKernelGGL((k_pkt<T, ADJ, 4>), grid, block, shm, stream, psi, z, ent, reg, a, gpart);
    }
    return hipGetLastError();
}

}  // namespace

int build_batch_packets(const std::vector<BatchPacketInst> &insts, const std::vector<PairOp> &ops,
                        const std::vector<uint32_t> &lists, BatchPackets &B) {
    B = BatchPackets{};
    std::vector<PacketPlan> plans(insts.size());
    FusedOpts o;
    o.es = 8;
    o.place_xcd = false;  // a batch launch mixes instances; its packets are not placed by XCD
    int R = 0;
    int64_t total_k = 0;
    for (size_t i = 0; i < insts.size(); ++i) {
        const BatchPacketInst &I = insts[i];
        if (I.nsa * I.nsb > packet_max_dim()) return fail(FSV_EINVAL, "internal: instance too large for packets");
        const std::vector<PairOp> pops(ops.begin() + I.off_ops, ops.begin() + I.off_ops + I.K);
        int rc = plan_packets(I.nsa, I.nsb, pops, lists, o, true, plans[i]);
        if (!rc) rc = check_packet_plan(plans[i], I.nsa * I.nsb, I.K);
        if (rc) return rc;
        R = std::max(R, (int)plans[i].groups.size());
        total_k = std::max<int64_t>(total_k, I.off_k + I.K);
    }
    B.runs = R;
    B.count.assign((size_t)total_k, 0);
    for (size_t i = 0; i < insts.size(); ++i)
        for (const FGroup &g : plans[i].groups) B.pstride = std::max(B.pstride, g.n_packets);
    B.pstride = std::max(B.pstride, 1);
    // launch r holds run r - (R - runs_i) of instance i (runs aligned at the end)
    for (int r = 0; r < R; ++r) {
        int wr = kPktHdr + 4;
        int npk = 0;
        for (size_t i = 0; i < insts.size(); ++i) {
            const int ri = r - (R - (int)plans[i].groups.size());
            if (ri < 0) continue;
            wr = std::max(wr, plans[i].groups[ri].wr);
            npk += plans[i].groups[ri].n_packets;
        }
        B.ent_off.push_back((int64_t)B.ent.size());
        B.reg_off.push_back((int64_t)B.reg.size());
        B.wr.push_back(wr);
        B.npk.push_back(npk);
        B.ent.resize(B.ent.size() + (size_t)npk * kPkt, kNone);
        B.reg.resize(B.reg.size() + (size_t)npk * wr, 0u);
        int64_t at = 0;
        for (size_t i = 0; i < insts.size(); ++i) {
            const int ri = r - (R - (int)plans[i].groups.size());
            if (ri < 0) continue;
            const BatchPacketInst &I = insts[i];
            const FGroup &g = plans[i].groups[ri];
            for (int k = g.k0; k < g.k0 + g.nops; ++k) B.count[(size_t)(I.off_k + k)] = g.n_packets;
            for (int q = 0; q < g.n_packets; ++q, ++at) {
                std::copy_n(plans[i].ent.begin() + g.ent_off + (int64_t)q * kPkt, kPkt,
                            B.ent.begin() + B.ent_off.back() + at * kPkt);
                uint32_t *h = &B.reg[(size_t)(B.reg_off.back() + at * wr)];
                std::copy_n(plans[i].reg.begin() + g.reg_off + (int64_t)q * g.wr, g.wr, h);
                const int64_t base = I.off_state;
                h[kBHdr] = (uint32_t)(base & 0xFFFFFFFF);
                h[kBHdr + 1] = (uint32_t)(base >> 32);
                h[kBHdr + 2] = (uint32_t)(I.nsa * I.nsb);
                h[kBHdr + 3] = (uint32_t)(I.off_k + g.k0);
                h[kBHdr + 4] = (uint32_t)g.nops;
                h[kBHdr + 5] = (uint32_t)q;
            }
        }
    }
    return FSV_OK;
}

size_t batch_packet_lds(int wr, bool adjoint) {
    return sizeof(double) * kPktScalars + (size_t)kPkt * (adjoint ? 2 : 1) * sizeof(double) + (size_t)wr * 4;
}

hipError_t launch_batch_packets(bool adjoint, double *arena, const uint32_t *ent, const uint32_t *reg, int wr,
                                int npk, const double *cs, double *gpart, int pstride, hipStream_t st) {
    if (npk <= 0) return hipSuccess;
    const dim3 grid((unsigned)std::min(npk, max_grid())), block(kWave);
    const size_t shm = batch_packet_lds(wr, adjoint);
    if (adjoint) {
        if (wr <= 4 * kWave * 2)
            hipLaunchKernelGGL((k_bpkt<true, 2>), grid, block, shm, st, arena, ent, reg, wr, npk, cs, gpart, pstride);
        else
            hipLaunchKernelGGL((k_bpkt<true, 4>), grid, block, shm, st, arena, ent, reg, wr, npk, cs, gpart, pstride);
    } else {
        if (wr <= 4 * kWave * 2)
            hipLaunchKernelGGL((k_bpkt<false, 2>), grid, block, shm, st, arena, ent, reg, wr, npk, cs, gpart, pstride);
        else
            hipLaunchKernelGGL((k_bpkt<false, 4>), grid, block, shm, st, arena, ent, reg, wr, npk, cs, gpart, pstride);
    }
    return hipGetLastError();
}

hipError_t launch_packets(int vtype, bool adjoint, void *state, const FusedSched &S, const FGroup &g,
                          const double *cs, double *gpart, int gstride, hipStream_t st, hipEvent_t t0,
                          hipEvent_t t1, bool store) {
    if (g.n_packets <= 0) {  // a run whose operators have no pairs here: no launch
        hipError_t e = hipSuccess;
        if (t0) e = hipEventRecord(t0, st);
        if (t1 && e == hipSuccess) e = hipEventRecord(t1, st);
        return e;
    }
    if (vtype == V_F64)
        return adjoint ? pkt_impl<double, true>(state, S, g, cs, gpart, gstride, st, t0, t1, store)
                       : pkt_impl<double, false>(state, S, g, cs, gpart, gstride, st, t0, t1, store);
    return adjoint ? pkt_impl<float, true>(state, S, g, cs, gpart, gstride, st, t0, t1, store)
                   : pkt_impl<float, false>(state, S, g, cs, gpart, gstride, st, t0, t1, store);
}

}  // namespace fsv
