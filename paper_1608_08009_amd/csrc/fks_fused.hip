// Fused FP32 collision kernel with FP64 conservation fix.
//
// Two work decompositions, chosen per call from the batch size:
//  * one workgroup per cell (large batches): a persistent workgroup takes cells
//    b, b + G, ..., evaluates every term of the cell, then sums the invariants
//    in FP64 across the workgroup, applies the fix and writes q_out / f_out
//    itself; its spectrum slot is reused from cell to cell.  One launch.
//  * pairs (small batches, twice the workgroups per cell), described next.
//
// Pair decomposition: two workgroups on the same XCD form a pair and share
// each of their cells; each workgroup evaluates half of the convolution terms
// of the cell (persistent loop over the pair's cells).  Both compute the
// forward transform and store the identical half spectrum in the cell's slot,
// which the pair then re-reads once per term from the XCD's L2 (the streaming
// reads of f and writes of partial sums are non-temporal so that they do not
// evict the reused spectrum slots and tables).  Each
// workgroup writes its partial sum; a second, HBM-bound kernel adds the two
// partials and applies the FP64 fix (the kernel boundary orders the writes,
// so no device-scope fence, which would flush the XCD's L2, is needed).
//   k_terms, per cell and workgroup:
//   1. f (FP64, HBM) -> FP32, forward 3D FFT, scale n^-3, zero the Nyquist
//      planes, store the half spectrum kz in [0, n/2) (eq. FC)
//   2. for each of its terms j (M*K gain terms, then the loss term (-L, 1)):
//      Z = (a_j + i b_j) fhat (mirror + conjugate for kz > n/2), inverse 3D
//      FFT, Q += Re(z) Im(z) in registers (eq. ode, fast form)
//   3. store the partial Q (FP32)
//   k_finish, per cell: Q = sum of the two partials, FP64 projection
//      lambda = G^{-1} C Q, Q_c = Q - C^T lambda, q_out = Q_c and/or
//      f_out = f_base + dt/tau Q_c (eqs. minim1, f_coll; f_base = f unless a
//      Runge-Kutta stage)
//
// Thread layouts (t = hi * n + lo, hi in [0, n/P), HP = n/P; pencil p in [0, P)):
//   C: pencil (y = hi + HP p, z = lo), registers over x      (physical side)
//   B: pencil (kx = kx_p, z = lo), registers over y
//   A: pencil (kx_p, ky_p), registers over kz                 (spectral side)
// With P = 2 a thread owns the mirrored pencils (kx, ky) and (-kx, -ky), so the
// tables and fhat (even and Hermitian in k) are loaded once per term for both.
// For hi = 0 the second pencil stands for the Nyquist pencil kx = n/2, which
// is zero: its A and B stages run on a duplicate of another pencil and its
// B -> C writes go to the unread padding column, so LDS row kx = n/2 keeps the
// zeros that the A -> B exchange left there (row ky = n/2 of every group is
// the zero Nyquist plane ky = n/2).
//
// Register budget (n = 32): a thread holds 2 x 32 complex values in flight and
// 64 accumulators; the scheduling fences keep the compiler from interleaving
// the per-pencil transforms, which would otherwise push the live set past 256
// VGPRs and spill the accumulators every term.  The own-pencil table and
// spectrum values of term j+1 are loaded during the last x transform of term j
// (software pipelining); the mirror-pencil values are loaded at the start of
// the term.  Tables and spectrum slots keep the planes kz = 2m and 2m + 1 side
// by side, so that each of these loads moves 16 bytes: the number of vector
// memory instructions, not their bytes, bounds the term loop (8-byte loads of
// the same data took 10% longer).
// Exchanges at n = 32 (two pencils per thread; B -> C in two rounds, four
// barriers): pencil 0's A -> B writes are spread over the sub-transforms of
// pencil 1's z transform and its reads over that transform's last combination;
// pencil 1's writes and reads likewise over pencil 0's y transform.  Round 0's
// B -> C writes of pencil 0 are spread over the sub-transforms of pencil 1's y
// transform, those of pencil 1 go out as its output groups are formed, and round 1's
// writes over the four sub-transforms of pencil 0's x transform, whose last
// combination then runs while round 1's reads are in flight, so that LDS traffic
// overlaps arithmetic instead of following it.
// LDS holds HP blocks of n rows with row stride n+1 (padding against bank
// conflicts; every LDS access is a per-thread base plus an immediate offset).
// A <-> B only swaps (lane, register) inside the n threads sharing hi: it goes
// through that group's own block (row = the pencil's ky, column = z) and needs
// no workgroup barrier when n divides 64 (the group lies in one wave); for
// n = 24 groups straddle waves and the exchange uses workgroup barriers.  B <-> C
// crosses waves: P rounds of n^3/P^2 values with workgroup barriers; in every
// round each group reads back only its own block, so the next group-local
// exchange can reuse that block without a barrier.  With one pencil per thread
// (n <= 24) the A -> B and B -> C writes go out as the z and y transforms' output
// groups are formed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "fks_common.hpp"

namespace fks {
namespace {

template <int N>
struct Cfg;
template <>
struct Cfg<8> { static constexpr int P = 1; };
template <>
struct Cfg<16> { static constexpr int P = 1; };
template <>
struct Cfg<24> { static constexpr int P = 1; };
template <>
struct Cfg<32> { static constexpr int P = 2; };

// ordering for the group-local A <-> B exchange: a group of n threads lies in
// one wave when n divides 64; otherwise (n = 24) groups straddle waves and the
// whole workgroup synchronises
template <int N>
__device__ __forceinline__ void group_sync();

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int N>
__device__ __forceinline__ void group_sync() {
    if constexpr (64 % N == 0) wave_sync();
    else __syncthreads();
}

// Hides a value from loop-invariant code motion so that per-thread address
// arithmetic is recomputed next to its loads instead of occupying registers
// for the whole kernel.
template <typename V>
__device__ __forceinline__ V opaque(V v) {
    asm volatile("" : "+v"(v));
    return v;
}

__device__ __forceinline__ cx<float> cmulf(cx<float> a, cx<float> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
__device__ __forceinline__ cx<float> cmulf_conj(cx<float> a, cx<float> b) {
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}

// spectral pencil (kx, ky) owned by thread (hi, lo) as pencil p
template <int N, int P>
__device__ __forceinline__ int kx_of(int p, int hi) {
    if (P == 1 || p == 0) return hi;
    return hi == 0 ? N / 2 : N - hi;
}
template <int N, int P>
__device__ __forceinline__ int ky_of(int p, int hi, int lo) {
    if (P == 1 || p == 0 || hi == 0) return lo;
    return (N - lo) % N;
}
// forward C -> B, round r: LDS block receiving spectral row x (the reader's hi)
template <int N, int P, int R, int X>
constexpr int fwd_block() {
    if constexpr (R == 0) return X;
    else return X == N / 2 ? 0 : N - X;
}

struct FusedArgs {
    const double* f;
    double* q_out;
    double* f_out;
    const double* f_base;   // state of the update (f unless a Runge-Kutta stage)
    int64_t ncell;
    double dt;
    const cx<float>* tab;   // [J][n/4][n][n][2] balanced (a, b), kz pairs adjacent
    int J;
    int npairs;
    cx<float>* fh;          // [ncell][n/4][n][n][2] (kz pairs adjacent)
    float* part;            // [ncell][2][n^3]
    const GridConst* gc;
    unsigned long long* guard;   // numeric guard word, or null
};

// Work queue over several segments of one n (an uneven batch): an item is a range of
// terms of one cell (cells with many terms are cut into nchunk ranges, so that no item
// is much longer than the rest); workgroups take items from one counter, largest items
// first.  Each item computes the cell's forward transform into the workgroup's slot,
// evaluates its terms and writes its FP32 partial sum; k_finish_q then adds a cell's
// partials and applies the FP64 fix.  Segments sit in the kernel arguments.
constexpr int kMaxQSeg = 16;
struct QSeg {
    const double* f;        // [ncell][n^3]
    const double* f_base;   // state of the update
    double* q_out;
    double* f_out;
    const cx<float>* tab;   // the plan's balanced FP32 tables, kz pairs adjacent
    const GridConst* gc;
    unsigned long long* guard;
    double dt;
    int64_t item0;          // first item of the segment (items are cell-major, then range)
    int64_t cell0;          // first cell of the segment in the finish grid
    int64_t part0;          // first partial slot (slot = part0 + item - item0)
    int J;
    int nchunk;
};
struct QueueArgs {
    QSeg seg[kMaxQSeg];
    int nseg;
    int64_t nitems;
    int64_t ncell;          // cells of all segments
    cx<float>* fh;          // [grid][n/4][n][n][2]: one spectrum slot per workgroup
    float* part;            // [slots][n^3]
    int* ctr;               // item counter, zero at launch
};

// the segment of a queue item (or of a finish cell): the last one whose first index is
// at most i; compile-time indices keep the argument table in scalar registers
template <bool BY_CELL>
__device__ __forceinline__ QSeg qseg_of(const QueueArgs& Q, int64_t i) {
    QSeg cur = Q.seg[0];
    sfor<kMaxQSeg>([&](auto sI) {
        constexpr int k = decltype(sI)::value;
        if constexpr (k > 0) {
            if (k < Q.nseg && (BY_CELL ? Q.seg[k].cell0 : Q.seg[k].item0) <= i) cur = Q.seg[k];
        }
    });
    return cur;
}

// MODE 0: the pair kernel above (partials, then k_finish).  MODE 1: one workgroup
// evaluates all terms of a cell and applies the FP64 fix and the update itself
// (persistent loop over cells b, b + G, ...; the spectrum slot is per workgroup and
// reused from cell to cell).  MODE 2: the work queue over several segments.
template <int MODE>
using TermsArgs = std::conditional_t<MODE == 2, QueueArgs, FusedArgs>;

template <int N, int MODE>
__global__ __launch_bounds__(N * N / Cfg<N>::P) void k_terms(TermsArgs<MODE> A) {
    constexpr bool ONE = MODE == 1;
    constexpr int P = Cfg<N>::P;
    constexpr int NT = N * N / P;
    constexpr int HP = N / P;
    constexpr int NN = N * N;
    constexpr int N3 = N * N * N;
    constexpr int RS = N + 1;        // LDS row stride (complex)
    constexpr int BS = N * RS;       // LDS block stride
    constexpr int HS = (N / 2) * N * N;      // spectrum slot per cell, and table stride per term
    __shared__ cx<float> lds[HP * BS];
    __shared__ double red[ONE ? 5 * (NT / 64) : 1];
    __shared__ int64_t s_item;

    const int t = threadIdx.x;
    const int hi = t / N, lo = t % N;
    cx<float>* const blk = lds + hi * BS;   // this group's block
    // pairs of workgroups on one XCD: blocks b and b ^ 8
    const int b = blockIdx.x;
    const int half = MODE == 0 ? (b >> 3) & 1 : 0;
    const int pair = MODE == 0 ? (b & 7) | ((b >> 4) << 3) : b;
    int64_t stride = 0;
    if constexpr (MODE != 2) stride = ONE ? (int64_t)gridDim.x : (int64_t)A.npairs;

    for (int64_t cell = pair, it = 0;; cell += stride, ++it) {
        const double* fc;
        const cx<float>* tab0;
        int Jt, j_begin, j_end;
        cx<float>* fh;
        float* mine = nullptr;   // partial sum of MODE 0 and 2
        if constexpr (MODE == 2) {
            if (t == 0) s_item = atomicAdd(A.ctr, 1);
            __syncthreads();
            const int64_t item = __builtin_amdgcn_readfirstlane(s_item);
            if (item >= A.nitems) break;
            const QSeg g = qseg_of<false>(A, item);
            const int64_t local = item - g.item0;
            const int64_t c = local / g.nchunk;
            const int k = (int)(local - c * g.nchunk);
            Jt = g.J;
            j_begin = (int)((int64_t)k * g.J / g.nchunk);
            j_end = (int)((int64_t)(k + 1) * g.J / g.nchunk);
            fc = g.f + c * (int64_t)N3;
            tab0 = g.tab;
            fh = A.fh + (int64_t)b * HS;
            mine = A.part + (g.part0 + local) * (int64_t)N3;
        } else {
            if (cell >= A.ncell) break;
            // split the terms in two; for odd J the extra term alternates between
            // the halves so that the pair stays on the same cell
            const int J0 = ONE ? A.J : (it & 1) ? A.J / 2 : (A.J + 1) / 2;
            j_begin = half ? J0 : 0;
            j_end = half ? A.J : J0;
            Jt = A.J;
            fc = A.f + cell * (int64_t)N3;
            tab0 = A.tab;
            fh = A.fh + (ONE ? (int64_t)b : cell) * (int64_t)HS;
            if constexpr (MODE == 0) mine = A.part + (cell * 2 + half) * (int64_t)N3;
        }

        // ---------------- forward transform ----------------
        cx<float> c[P][N];
        sfor<P>([&](auto pI) {
            constexpr int p = decltype(pI)::value;
            const double* src = fc + opaque((hi + HP * p) * N + lo);
            sfor<N>([&](auto xI) {
                constexpr int x = decltype(xI)::value;
                c[p][x] = cx<float>{(float)__builtin_nontemporal_load(src + x * NN), 0.0f};
            });
            fft<float, N, -1>(c[p]);
        });
        cx<float> bb[P][N];
        sfor<P>([&](auto rI) {   // C -> B, round r delivers B-pencil r
            constexpr int r = decltype(rI)::value;
            __syncthreads();
            sfor<P>([&](auto pI) {
                constexpr int p = decltype(pI)::value;
                cx<float>* dst = lds + (hi + HP * p) * RS + lo;   // row y, column z
                sfor<HP>([&](auto xI) {
                    constexpr int x = HP * r + decltype(xI)::value;
                    dst[fwd_block<N, P, r, x>() * BS] = c[p][x];
                });
            });
            __syncthreads();
            sfor<N>([&](auto yI) {
                constexpr int y = decltype(yI)::value;
                bb[r][y] = blk[y * RS + lo];
            });
        });
        sfor<P>([&](auto pI) {
            constexpr int p = decltype(pI)::value;
            fft<float, N, -1>(bb[p]);
            // B -> A inside the group: element (row ky, column z)
            sfor<N>([&](auto kI) {
                constexpr int ky = decltype(kI)::value;
                blk[ky * RS + lo] = bb[p][ky];
            });
            group_sync<N>();
            cx<float> a[N];
            const cx<float>* arow = blk + ky_of<N, P>(p, hi, lo) * RS;   // this pencil's actual ky
            sfor<N>([&](auto zI) {
                constexpr int z = decltype(zI)::value;
                a[z] = arow[z];
            });
            group_sync<N>();
            fft<float, N, -1>(a);
            const int kx = kx_of<N, P>(p, hi), ky = ky_of<N, P>(p, hi, lo);
            const float s = ((kx == N / 2) || (ky == N / 2)) ? 0.0f : 1.0f / (float)N3;
            // kz pairs (2m, 2m + 1) adjacent, so that one 16-byte access moves two planes
            float4* o = reinterpret_cast<float4*>(fh) + opaque(kx * N + ky);
            sfor<N / 4>([&](auto mI) {
                constexpr int m = decltype(mI)::value;
                o[m * NN] = float4{a[2 * m].x * s, a[2 * m].y * s, a[2 * m + 1].x * s, a[2 * m + 1].y * s};
            });
        });
        __threadfence_block();
        __syncthreads();

        // ---------------- this workgroup's terms ----------------
        float q[P][N];
        sfor<P>([&](auto pI) {
            constexpr int p = decltype(pI)::value;
            sfor<N>([&](auto xI) { q[p][decltype(xI)::value] = 0.0f; });
        });
        // Table and spectrum at pencil (kx, ky), kz in [0, n/2), as n/4 loads of 16 bytes
        // (kz pairs are adjacent in both; a wave's load covers 1 KiB of consecutive
        // memory).  Half as many load instructions as 8-byte loads of the same bytes:
        // the issue of vector memory instructions, not their bytes, limits this loop.
        auto load_pairs = [&](auto m0I, auto m1I, const char* tj, uint32_t o16, cx<float>* t, cx<float>* f) {
            constexpr int M0 = decltype(m0I)::value, M1 = decltype(m1I)::value;
            sfor<M1 - M0>([&](auto mI) {
                constexpr int m = M0 + decltype(mI)::value;
                constexpr uint32_t zo = m * NN * sizeof(float4);
                const float4 a = *(const float4*)(tj + (o16 + zo));
                const float4 c = *(const float4*)((const char*)fh + (o16 + zo));
                t[2 * m] = {a.x, a.y};
                t[2 * m + 1] = {a.z, a.w};
                f[2 * m] = {c.x, c.y};
                f[2 * m + 1] = {c.z, c.w};
            });
        };
        // own pencil (hi, lo): loaded one term ahead, during the last x transform of the
        // previous term
        cx<float> pt[N / 2], pf[N / 2];
        auto load_own = [&](int jj) {
            load_pairs(std::integral_constant<int, 0>{}, std::integral_constant<int, N / 4>{},
                       (const char*)(tab0 + (size_t)jj * HS), uint32_t(opaque(hi * N + lo)) * 16u, pt, pf);
        };
        load_own(min(j_begin, Jt - 1));
        for (int j = j_begin; j < j_end; ++j) {
            const cx<float>* tj = tab0 + (size_t)j * HS;
            cx<float> za[P][N];
            // Products Z = (a + i b) fhat.  Own pencil (hi, lo), kz in [0, n/2): from the
            // prefetched pt, pf; mirror pencil (-hi, -lo): loaded here in NG groups of kz
            // pairs, each group's loads issued one phase before its products, so that part
            // of the loads is in flight while the previous part is consumed (all at once, or
            // as the compiler orders them by itself, is slower).
            const uint32_t ob16 = uint32_t(opaque(((N - hi) % N) * N + ((N - lo) % N))) * 16u;
            cx<float> mt[N / 2], mf[N / 2];
            constexpr int NPR = N / 4;   // kz pairs
            constexpr int NG = NPR % 4 == 0 ? 4 : NPR % 3 == 0 ? 3 : 2;
            constexpr int GS = (N / 2) / NG;   // kz per group
            static_assert(GS * NG == N / 2 && GS % 2 == 0, "mirror load groups");
            // pencil 0 = (hi, lo): kz from (hi, lo), -kz from the mirror (conjugated);
            // pencil 1 = (-hi, -lo): kz from the mirror, -kz from (hi, lo)
            auto own_products = [&](auto kI) {
                constexpr int kz = decltype(kI)::value;
                za[0][kz] = cmulf(pt[kz], pf[kz]);
                if constexpr (P == 2 && kz > 0) za[1][N - kz] = cmulf_conj(pt[kz], pf[kz]);
            };
            auto mirror_products = [&](auto kI) {
                constexpr int kz = decltype(kI)::value;
                if constexpr (kz > 0) za[0][N - kz] = cmulf_conj(mt[kz], mf[kz]);
                if constexpr (P == 2) za[1][kz] = cmulf(mt[kz], mf[kz]);
            };
            sfor<NG + 1>([&](auto phI) {
                constexpr int ph = decltype(phI)::value;
                if constexpr (ph < NG)
                    load_pairs(std::integral_constant<int, ph * GS / 2>{}, std::integral_constant<int, (ph + 1) * GS / 2>{},
                               (const char*)tj, ob16, mt, mf);
                if constexpr (ph == 0) sfor<N / 2>([&](auto kI) { own_products(kI); });
                if constexpr (ph > 0)
                    sfor<GS>([&](auto kI) { mirror_products(std::integral_constant<int, (ph - 1) * GS + decltype(kI)::value>{}); });
                __builtin_amdgcn_sched_barrier(0);
            });
            za[0][N / 2] = cx<float>{0.0f, 0.0f};
            if constexpr (P == 2) {
                za[1][N / 2] = cx<float>{0.0f, 0.0f};
            }
            cx<float> zb[P][N];
            if constexpr (P == 2) {
                // z transforms and A -> B of two pencils: pencil 0's writes go out between the
                // sub-transforms of pencil 1's z transform and its reads between that
                // transform's output groups; pencil 1's writes and reads likewise during
                // pencil 0's y transform (the group lies in one wave, whose LDS accesses are
                // served in order, so the reads see every write issued before them)
                constexpr int NSUB = first_radix<N>(), NCMB = N / NSUB;
                auto a_put = [&](auto pI, auto z0I, auto z1I) {
                    constexpr int p = decltype(pI)::value;
                    constexpr int Z0 = decltype(z0I)::value, Z1 = decltype(z1I)::value;
                    cx<float>* arow = blk + ky_of<N, P>(p, hi, lo) * RS;   // row = this pencil's actual ky
                    sfor<Z1 - Z0>([&](auto zI) {
                        constexpr int z = Z0 + decltype(zI)::value;
                        arow[z] = za[p][z];
                    });
                };
                auto b_get = [&](auto pI, auto k0I, auto k1I) {
                    constexpr int p = decltype(pI)::value;
                    constexpr int K0 = decltype(k0I)::value, K1 = decltype(k1I)::value;
                    sfor<K1 - K0>([&](auto kI) {
                        constexpr int ky = K0 + decltype(kI)::value;
                        zb[p][ky] = blk[ky * RS + lo];
                    });
                };
                auto exchange = [&](auto pI, auto iI) {
                    constexpr int i = decltype(iI)::value;
                    __builtin_amdgcn_sched_barrier(0);
                    if constexpr (i < NSUB) {
                        a_put(pI, std::integral_constant<int, N * i / NSUB>{},
                              std::integral_constant<int, N * (i + 1) / NSUB>{});
                        if constexpr (i == NSUB - 1) group_sync<N>();
                    } else {
                        constexpr int k = i - NSUB;
                        b_get(pI, std::integral_constant<int, N * k / NCMB>{},
                              std::integral_constant<int, N * (k + 1) / NCMB>{});
                    }
                    __builtin_amdgcn_sched_barrier(0);
                };
                __builtin_amdgcn_sched_barrier(0);
                fft<float, N, 1>(za[0]);
                fft_hook<float, N, 1>(za[1], [&](auto iI) { exchange(std::integral_constant<int, 0>{}, iI); });
                fft_hook<float, N, 1>(zb[0], [&](auto iI) { exchange(std::integral_constant<int, 1>{}, iI); });
                group_sync<N>();
            } else {
                // one pencil: the z transform with the A -> B writes of its output groups (a
                // group that straddles waves must not overwrite its block before all of its
                // threads have read their columns of the previous B -> C round), then the reads
                if constexpr (64 % N != 0) __syncthreads();
                constexpr int R1 = first_radix<N>(), M1 = N / R1;
                cx<float>* arow = blk + ky_of<N, P>(0, hi, lo) * RS;   // row = this pencil's actual ky
                __builtin_amdgcn_sched_barrier(0);
                fft_hook<float, N, 1>(za[0], [&](auto iI) {
                    constexpr int i = decltype(iI)::value;
                    if constexpr (i >= R1) {   // output group i - R1: z = i - R1 + M1 q
                        __builtin_amdgcn_sched_barrier(0);
                        sfor<R1>([&](auto qI) {
                            constexpr int z = i - R1 + M1 * decltype(qI)::value;
                            arow[z] = za[0][z];
                        });
                        __builtin_amdgcn_sched_barrier(0);
                    }
                });
                group_sync<N>();
                sfor<N>([&](auto kI) {
                    constexpr int ky = decltype(kI)::value;
                    zb[0][ky] = blk[ky * RS + lo];
                });
            }
            cx<float> zc[P][N];
            if constexpr (P == 2) {
                // B -> C writes of pencil p, round r, y offset yy in [Y0, Y1)
                auto put = [&](auto pI, auto rI, auto y0I, auto y1I) {
                    constexpr int p = decltype(pI)::value;
                    constexpr int r = decltype(rI)::value;
                    constexpr int Y0 = decltype(y0I)::value, Y1 = decltype(y1I)::value;
                    cx<float>* dst = lds + ((p == 1 && hi == 0) ? lo * RS + N : kx_of<N, P>(p, hi) * RS + lo);
                    sfor<Y1 - Y0>([&](auto yI) {
                        constexpr int yy = Y0 + decltype(yI)::value;
                        dst[yy * BS] = zb[p][HP * r + yy];
                    });
                };
                auto get = [&](auto rI) {
                    constexpr int r = decltype(rI)::value;
                    sfor<N>([&](auto kI) {
                        constexpr int kx = decltype(kI)::value;
                        zc[r][kx] = blk[kx * RS + lo];
                    });
                };
                auto acc = [&](auto pI) {
                    constexpr int p = decltype(pI)::value;
                    sfor<N>([&](auto xI) {
                        constexpr int x = decltype(xI)::value;
                        q[p][x] = fmaf(zc[p][x].x, zc[p][x].y, q[p][x]);
                    });
                };
                using I0 = std::integral_constant<int, 0>;
                using I1 = std::integral_constant<int, 1>;
                __builtin_amdgcn_sched_barrier(0);
                __syncthreads();
                // round 0: pencil 0's writes spread over the sub-transforms of pencil 1's y
                // transform, and pencil 1's own writes issued as its output groups come out
                // (group k holds y = k + M q, of which k and k + M belong to round 0)
                constexpr int NSUBY = first_radix<N>(), MY = N / NSUBY;
                static_assert(HP == 2 * MY, "round 0 takes two outputs of every group");
                fft_hook<float, N, 1>(zb[1], [&](auto iI) {
                    constexpr int i = decltype(iI)::value;
                    __builtin_amdgcn_sched_barrier(0);
                    if constexpr (i < NSUBY) {
                        put(I0{}, I0{}, std::integral_constant<int, HP * i / NSUBY>{},
                            std::integral_constant<int, HP * (i + 1) / NSUBY>{});
                    } else {
                        constexpr int k = i - NSUBY;
                        put(I1{}, I0{}, std::integral_constant<int, k>{}, std::integral_constant<int, k + 1>{});
                        put(I1{}, I0{}, std::integral_constant<int, k + MY>{}, std::integral_constant<int, k + MY + 1>{});
                    }
                    __builtin_amdgcn_sched_barrier(0);
                });
                __syncthreads();
                get(I0{});
                __syncthreads();
                // round 1: the writes spread over the first-level sub-transforms of pencil 0's
                // x transform, then the barrier, then the reads overlap its last combination
                constexpr int NSUB = first_radix<N>();
                fft_hook<float, N, 1>(zc[0], [&](auto iI) {
                    constexpr int i = decltype(iI)::value;
                    if constexpr (i < NSUB) {
                        __builtin_amdgcn_sched_barrier(0);
                        constexpr int w0 = 2 * HP * i / NSUB, w1 = 2 * HP * (i + 1) / NSUB;
                        // w in [w0, w1): pencil w / HP, y offset w % HP (ranges stay in one pencil)
                        static_assert((w0 / HP) == ((w1 - 1) / HP), "write range crosses pencils");
                        put(std::integral_constant<int, w0 / HP>{}, I1{}, std::integral_constant<int, w0 % HP>{},
                            std::integral_constant<int, (w1 - 1) % HP + 1>{});
                        __builtin_amdgcn_sched_barrier(0);
                    }
                    if constexpr (i == NSUB - 1) {
                        __syncthreads();
                        get(I1{});
                        __builtin_amdgcn_sched_barrier(0);
                    }
                });
                acc(I0{});
                __builtin_amdgcn_sched_barrier(0);
                load_own(min(j + 1, j_end - 1));
                __builtin_amdgcn_sched_barrier(0);
                fft<float, N, 1>(zc[1]);
                acc(I1{});
            } else {
                // one B -> C round: row kx = hi, column z = lo of every y block, written as the
                // y transform's output groups come out (every group has read its own block by
                // the barrier), then the C pencil (y = hi, z = lo) from the own block
                __syncthreads();
                constexpr int R1 = first_radix<N>(), M1 = N / R1;
                cx<float>* dst = lds + hi * RS + lo;
                fft_hook<float, N, 1>(zb[0], [&](auto iI) {
                    constexpr int i = decltype(iI)::value;
                    if constexpr (i >= R1) {   // output group i - R1: y = i - R1 + M1 q
                        __builtin_amdgcn_sched_barrier(0);
                        sfor<R1>([&](auto qI) {
                            constexpr int yy = i - R1 + M1 * decltype(qI)::value;
                            dst[yy * BS] = zb[0][yy];
                        });
                        __builtin_amdgcn_sched_barrier(0);
                    }
                });
                __syncthreads();
                sfor<N>([&](auto kI) {
                    constexpr int kx = decltype(kI)::value;
                    zc[0][kx] = blk[kx * RS + lo];
                });
                __builtin_amdgcn_sched_barrier(0);   // next term's own-pencil loads overlap the transform
                load_own(min(j + 1, j_end - 1));
                __builtin_amdgcn_sched_barrier(0);
                fft<float, N, 1>(zc[0]);
                sfor<N>([&](auto xI) {
                    constexpr int x = decltype(xI)::value;
                    q[0][x] = fmaf(zc[0][x].x, zc[0][x].y, q[0][x]);
                });
            }
        }

        if constexpr (ONE) {
            // ---------------- FP64 fix and update (C layout: x, y = hi + HP p, z = lo) ----------------
            // thread coordinates re-derived here so that nothing computed before the term
            // loop stays live across it (the loop needs every register)
            const int t = opaque((int)threadIdx.x);
            const int hi = t / N, lo = t % N;
            const double h = A.gc->dv / A.gc->T;
            const double uz = -1.0 + lo * h;
            double m[5] = {0, 0, 0, 0, 0};
            sfor<P>([&](auto pI) {
                constexpr int p = decltype(pI)::value;
                const double uy = -1.0 + (hi + HP * p) * h;
                const double ryz = fma(uy, uy, uz * uz);
                sfor<N>([&](auto xI) {
                    constexpr int x = decltype(xI)::value;
                    const double ux = -1.0 + x * h;
                    const double qq = (double)q[p][x];
                    m[0] += qq;
                    m[1] = fma(qq, ux, m[1]);
                    m[2] = fma(qq, uy, m[2]);
                    m[3] = fma(qq, uz, m[3]);
                    m[4] = fma(qq, fma(ux, ux, ryz), m[4]);
                });
            });
            block_sum5<NT>(m, red);
            if (A.guard && t == 0 && !isfinite(m[0] + m[1] + m[2] + m[3] + m[4]))
                atomicMin(A.guard, (unsigned long long)cell);
            double lam[5];
            solve5(*A.gc, m, lam);
            sfor<P>([&](auto pI) {   // one pencil at a time (register budget)
                constexpr int p = decltype(pI)::value;
                __builtin_amdgcn_sched_barrier(0);
                // recomputed, not kept live across the reduction: the node coordinates
                // and the FP64 copies of q of the moment sums
                const double h = opaque(A.gc->dv / A.gc->T);
                const double uz = -1.0 + lo * h;
                const double uy = -1.0 + (hi + HP * p) * h;
                const double lyz = fma(lam[4], fma(uy, uy, uz * uz), fma(lam[2], uy, fma(lam[3], uz, lam[0])));
                const int64_t row = cell * (int64_t)N3 + (hi + HP * p) * N + lo;
                auto qc = [&](auto xI) {
                    constexpr int x = decltype(xI)::value;
                    const double ux = -1.0 + x * h;
                    return (double)opaque(q[p][x]) - fma(lam[4], ux * ux, fma(lam[1], ux, lyz));
                };
                if (A.f_out) {
                    // every load of the pencil before its first store: f_out may alias f_base
                    double fb[N];
                    sfor<N>([&](auto xI) {
                        constexpr int x = decltype(xI)::value;
                        fb[x] = __builtin_nontemporal_load(A.f_base + row + x * NN);
                    });
                    sfor<N>([&](auto xI) {
                        constexpr int x = decltype(xI)::value;
                        const double v = qc(xI);
                        if (A.q_out) __builtin_nontemporal_store(v, A.q_out + row + x * NN);
                        __builtin_nontemporal_store(fma(A.dt, v, fb[x]), A.f_out + row + x * NN);
                    });
                } else {
                    sfor<N>([&](auto xI) {
                        constexpr int x = decltype(xI)::value;
                        __builtin_nontemporal_store(qc(xI), A.q_out + row + x * NN);
                    });
                }
            });
        } else {
            // ---------------- partial sum (C layout: x, y = hi + HP p, z = lo) ----------------
            sfor<P>([&](auto pI) {
                constexpr int p = decltype(pI)::value;
                float* o = mine + opaque((hi + HP * p) * N + lo);
                sfor<N>([&](auto xI) {
                    constexpr int x = decltype(xI)::value;
                    __builtin_nontemporal_store(q[p][x], o + x * NN);
                });
            });
        }
    }
}

// Sum of the two partials, FP64 projection onto the kernel of the collision
// invariants and the update; one workgroup per cell, values kept in registers.
// Thread t owns VW = 4 consecutive nodes in z starting at node 4 t + 4 FT k
// (16-byte partial loads, 32-byte f loads and stores): its (y, z) are fixed
// and x advances by 4 FT / n^2 per step.
template <int N>
constexpr int finish_threads() {
    if constexpr (N == 24) return 576;   // a multiple of 64 and of n^2/4 that divides n^3/4
    else return N * N * N / 4 < 512 ? N * N * N / 4 : 512;
}

typedef float f4v __attribute__((ext_vector_type(4)));
typedef double d2v __attribute__((ext_vector_type(2)));

template <int N>
__global__ __launch_bounds__(finish_threads<N>()) void k_finish(FusedArgs A) {
    constexpr int N3 = N * N * N;
    constexpr int VW = 4;
    constexpr int FT = finish_threads<N>();
    constexpr int V = N3 / (FT * VW);        // vectors per thread
    constexpr int XS = FT * VW / (N * N);    // x advance per step
    static_assert(V * FT * VW == N3 && XS * N * N == FT * VW, "finish layout");
    __shared__ double red[5 * (FT / 64)];
    const int t = threadIdx.x;
    const int64_t cell = blockIdx.x;
    const float* p0 = A.part + cell * 2 * (int64_t)N3;
    const float* p1 = p0 + N3;
    const double h = A.gc->dv / A.gc->T;
    const int z0 = (VW * t) % N, y = (VW * t / N) % N, x0 = VW * t / (N * N);
    const double uy = -1.0 + y * h;
    double uz[VW];
#pragma unroll
    for (int c = 0; c < VW; ++c) uz[c] = -1.0 + (z0 + c) * h;
    double qv[V][VW];
    double m[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < V; ++k) {
        const int i = VW * t + k * FT * VW;
        const double ux = -1.0 + (x0 + k * XS) * h;
        const f4v a = __builtin_nontemporal_load((const f4v*)(p0 + i));
        const f4v b = __builtin_nontemporal_load((const f4v*)(p1 + i));
        const double rxy = fma(ux, ux, uy * uy);
#pragma unroll
        for (int c = 0; c < VW; ++c) {
            const double q = (double)a[c] + (double)b[c];
            qv[k][c] = q;
            m[0] += q;
            m[1] = fma(q, ux, m[1]);
            m[2] = fma(q, uy, m[2]);
            m[3] = fma(q, uz[c], m[3]);
            m[4] = fma(q, fma(uz[c], uz[c], rxy), m[4]);
        }
    }
    block_sum5<FT>(m, red);
    if (A.guard && t == 0 && !isfinite(m[0] + m[1] + m[2] + m[3] + m[4])) atomicMin(A.guard, (unsigned long long)cell);
    double lam[5];
    solve5(*A.gc, m, lam);
    const int64_t base = cell * (int64_t)N3 + VW * t;
#pragma unroll
    for (int k = 0; k < V; ++k) {
        const double ux = -1.0 + (x0 + k * XS) * h;
        const double lx = fma(lam[4], fma(ux, ux, uy * uy), fma(lam[1], ux, fma(lam[2], uy, lam[0])));
#pragma unroll
        for (int c = 0; c < VW; ++c) qv[k][c] -= fma(lam[4], uz[c] * uz[c], fma(lam[3], uz[c], lx));
    }
    if (A.q_out) {
#pragma unroll
        for (int k = 0; k < V; ++k) {
            d2v* o = (d2v*)(A.q_out + base + k * FT * VW);
            __builtin_nontemporal_store(d2v{qv[k][0], qv[k][1]}, o);
            __builtin_nontemporal_store(d2v{qv[k][2], qv[k][3]}, o + 1);
        }
    }
    if (A.f_out) {
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const d2v* fi = (const d2v*)(A.f_base + base + k * FT * VW);
            d2v* o = (d2v*)(A.f_out + base + k * FT * VW);
            const d2v f0 = __builtin_nontemporal_load(fi), f1 = __builtin_nontemporal_load(fi + 1);
            __builtin_nontemporal_store(d2v{fma(A.dt, qv[k][0], f0[0]), fma(A.dt, qv[k][1], f0[1])}, o);
            __builtin_nontemporal_store(d2v{fma(A.dt, qv[k][2], f1[0]), fma(A.dt, qv[k][3], f1[1])}, o + 1);
        }
    }
}

// Finish of the work queue: one workgroup per cell of all segments; sums the cell's nchunk
// FP32 partials in FP64 (fixed order: bit-reproducible), then the FP64 fix and update
// as in k_finish.
template <int N>
__global__ __launch_bounds__(finish_threads<N>()) void k_finish_q(QueueArgs Q) {
    constexpr int N3 = N * N * N;
    constexpr int VW = 4;
    constexpr int FT = finish_threads<N>();
    constexpr int V = N3 / (FT * VW);
    constexpr int XS = FT * VW / (N * N);
    __shared__ double red[5 * (FT / 64)];
    const int t = threadIdx.x;
    const int64_t gcell = blockIdx.x;
    const QSeg g = qseg_of<true>(Q, gcell);
    const int64_t c = gcell - g.cell0;
    const float* p0 = Q.part + (g.part0 + c * g.nchunk) * (int64_t)N3;
    const double h = g.gc->dv / g.gc->T;
    const int z0 = (VW * t) % N, y = (VW * t / N) % N, x0 = VW * t / (N * N);
    const double uy = -1.0 + y * h;
    double uz[VW];
#pragma unroll
    for (int k = 0; k < VW; ++k) uz[k] = -1.0 + (z0 + k) * h;
    double qv[V][VW];
    double m[5] = {0, 0, 0, 0, 0};
#pragma unroll
    for (int k = 0; k < V; ++k) {
        const int i = VW * t + k * FT * VW;
        f4v a = __builtin_nontemporal_load((const f4v*)(p0 + i));
        double acc[VW] = {(double)a[0], (double)a[1], (double)a[2], (double)a[3]};
        for (int r = 1; r < g.nchunk; ++r) {
            a = __builtin_nontemporal_load((const f4v*)(p0 + (int64_t)r * N3 + i));
#pragma unroll
            for (int e = 0; e < VW; ++e) acc[e] += (double)a[e];
        }
        const double ux = -1.0 + (x0 + k * XS) * h;
        const double rxy = fma(ux, ux, uy * uy);
#pragma unroll
        for (int e = 0; e < VW; ++e) {
            const double q = acc[e];
            qv[k][e] = q;
            m[0] += q;
            m[1] = fma(q, ux, m[1]);
            m[2] = fma(q, uy, m[2]);
            m[3] = fma(q, uz[e], m[3]);
            m[4] = fma(q, fma(uz[e], uz[e], rxy), m[4]);
        }
    }
    block_sum5<FT>(m, red);
    if (g.guard && t == 0 && !isfinite(m[0] + m[1] + m[2] + m[3] + m[4])) atomicMin(g.guard, (unsigned long long)c);
    double lam[5];
    solve5(*g.gc, m, lam);
    const int64_t base = c * (int64_t)N3 + VW * t;
#pragma unroll
    for (int k = 0; k < V; ++k) {
        const double ux = -1.0 + (x0 + k * XS) * h;
        const double lx = fma(lam[4], fma(ux, ux, uy * uy), fma(lam[1], ux, fma(lam[2], uy, lam[0])));
#pragma unroll
        for (int e = 0; e < VW; ++e) qv[k][e] -= fma(lam[4], uz[e] * uz[e], fma(lam[3], uz[e], lx));
    }
    if (g.q_out) {
#pragma unroll
        for (int k = 0; k < V; ++k) {
            d2v* o = (d2v*)(g.q_out + base + k * FT * VW);
            __builtin_nontemporal_store(d2v{qv[k][0], qv[k][1]}, o);
            __builtin_nontemporal_store(d2v{qv[k][2], qv[k][3]}, o + 1);
        }
    }
    if (g.f_out) {
#pragma unroll
        for (int k = 0; k < V; ++k) {
            const d2v* fi = (const d2v*)(g.f_base + base + k * FT * VW);
            d2v* o = (d2v*)(g.f_out + base + k * FT * VW);
            const d2v f0 = __builtin_nontemporal_load(fi), f1 = __builtin_nontemporal_load(fi + 1);
            __builtin_nontemporal_store(d2v{fma(g.dt, qv[k][0], f0[0]), fma(g.dt, qv[k][1], f0[1])}, o);
            __builtin_nontemporal_store(d2v{fma(g.dt, qv[k][2], f1[0]), fma(g.dt, qv[k][3], f1[1])}, o + 1);
        }
    }
}

__global__ void k_zero_counter(int* ctr) {
    if (threadIdx.x == 0) *ctr = 0;
}

template <int N>
int grid_for(int device) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0)
        cus = 256;
    int per = 0;
    constexpr int NT = N * N / Cfg<N>::P;
    int per1 = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_terms<N, 0>, NT, 0) != hipSuccess || per <= 0) per = 1;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per1, k_terms<N, 1>, NT, 0) != hipSuccess || per1 <= 0) per1 = 1;
    per = std::min(per, per1);
    int g = cus * per;
    return std::max(16, (g / 16) * 16);   // whole XCD pairs: multiple of 16 workgroups
}

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

struct WsLayout {
    size_t fh, part, total;
};
// pairs of workgroups actually launched: a multiple of 8, at most grid/2
inline int npairs_for(const fks_plan* p, int64_t ncell) {
    const int maxp = p->fused_grid / 2;
    int64_t want = std::min<int64_t>(ncell, maxp);
    return (int)std::max<int64_t>(8, ((want + 7) / 8) * 8 > maxp ? (maxp / 8) * 8 : ((want + 7) / 8) * 8);
}

// Choice between the two decompositions, in units of one term of one cell on
// one workgroup.  One workgroup per cell: ceil(ncell / G) rounds of J terms
// plus the forward transform (about one term).  Pairs: rounds of half the
// terms plus a forward transform each, and the separate finish kernel, which
// costs about three terms per G cells (n = 32: 0.61 ms for 4096 cells against
// 11 us per term and round).  Small batches favour pairs (twice the
// workgroups per cell), large ones one workgroup per cell (one forward
// transform and no partial sums in HBM).
inline bool one_per_cell(const fks_plan* p, int64_t ncell) {
    if (ncell <= 0) return false;
    const Schedule sc = schedule_for(p, ncell);   // measured by fks_autotune
    if (sc.one >= 0) return sc.one == 1;
    const int64_t G = p->fused_grid;
    const int64_t J = p->J;
    const int64_t c1 = (ncell + G - 1) / G * (J + 1);
    const int64_t np = npairs_for(p, ncell);
    const int64_t c2 = (ncell + np - 1) / np * ((J + 1) / 2 + 1) + 3 * ((ncell + G - 1) / G);
    return c1 <= c2;
}

inline int64_t one_grid(const fks_plan* p, int64_t ncell) { return std::min<int64_t>(p->fused_grid, ncell); }

// Workspace: the pair kernels keep one spectrum slot per cell plus two FP32
// partial sums per cell; one workgroup per cell needs one slot per workgroup.
inline WsLayout ws_layout(const fks_plan* p, int64_t ncell) {
    const int n = p->desc.n;
    WsLayout w{};
    const size_t n3 = (size_t)n * n * n;
    const size_t slot = (size_t)(n / 2) * n * n * sizeof(cx<float>);
    w.fh = 0;
    if (one_per_cell(p, ncell)) {
        w.part = align256((size_t)one_grid(p, ncell) * slot);
        w.total = w.part;
        return w;
    }
    w.part = align256((size_t)ncell * slot);
    w.total = w.part + align256((size_t)ncell * 2 * n3 * sizeof(float));
    return w;
}

// event timing (off by default): events 0..2 bracket k_terms and k_finish (0..1
// bracket the single kernel of the one-workgroup-per-cell decomposition)
struct Prof {
    bool on = false;
    bool made = false;
    int device = -1;
    int count = 0;
    hipEvent_t ev[3];
};
Prof g_prof;

hipError_t prof_mark(int i, hipStream_t st) {
    if (!g_prof.on) return hipSuccess;
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (!g_prof.made || g_prof.device != dev) {
        if (g_prof.made)
            for (auto& x : g_prof.ev) (void)hipEventDestroy(x);
        g_prof.made = false;
        for (auto& x : g_prof.ev)
            if ((e = hipEventCreate(&x)) != hipSuccess) return e;
        g_prof.made = true;
        g_prof.device = dev;
    }
    g_prof.count = i;
    return hipEventRecord(g_prof.ev[i], st);
}

template <int N>
hipError_t launch(const fks_plan* p, const fks_segment& s, void* ws, hipStream_t st) {
    constexpr int NT = N * N / Cfg<N>::P;
    const WsLayout w = ws_layout(p, s.ncell);
    const bool one = one_per_cell(p, s.ncell);
    char* base = (char*)ws;
    FusedArgs a{};
    a.f = s.f;
    a.q_out = s.q_out;
    a.f_out = s.f_out;
    a.f_base = s.f_base ? s.f_base : s.f;
    a.ncell = s.ncell;
    a.dt = s.dt_over_tau;
    a.tab = reinterpret_cast<const cx<float>*>(p->d_tab32p);
    a.J = p->J;
    a.npairs = npairs_for(p, s.ncell);
    a.fh = reinterpret_cast<cx<float>*>(base + w.fh);
    a.part = reinterpret_cast<float*>(base + w.part);
    a.gc = p->d_gc;
    a.guard = p->d_guard;
    hipError_t e = prof_mark(0, st);
    if (e != hipSuccess) return e;
    if (one) {
        k_terms<N, 1><<<(unsigned)one_grid(p, s.ncell), NT, 0, st>>>(a);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        return prof_mark(1, st);
    }
    k_terms<N, 0><<<(unsigned)(2 * a.npairs), NT, 0, st>>>(a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = prof_mark(1, st)) != hipSuccess) return e;
    k_finish<N><<<(unsigned)s.ncell, finish_threads<N>(), 0, st>>>(a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return prof_mark(2, st);
}

// Work-queue plan of several segments of one n: cells whose term count is much larger
// than the average item get cut into nchunk term ranges (about four items per resident
// workgroup, no range shorter than four terms), and segments are ordered by item length,
// longest first.
struct QueuePlan {
    int nseg = 0;
    int order[kMaxQSeg];
    int nchunk[kMaxQSeg];
    int64_t items = 0, slots = 0, cells = 0;
};
QueuePlan queue_plan(const fks_segment* const* g, int nseg) {
    QueuePlan q;
    q.nseg = nseg;
    const int64_t G = g[0]->plan->fused_grid;
    // items per resident workgroup: the direction batch of an item is about J / (that many
    // items per cell); the first segment's plan carries the autotuner's choice
    const int64_t ipw = g[0]->plan->queue_ipw > 0 ? g[0]->plan->queue_ipw : 4;
    int64_t units = 0;
    for (int i = 0; i < nseg; ++i) units += g[i]->ncell * (g[i]->plan->J + 1);
    const int64_t len = std::max<int64_t>(4, (units + ipw * G - 1) / (ipw * G));
    for (int i = 0; i < nseg; ++i) {
        const int J = g[i]->plan->J;
        q.nchunk[i] = (int)std::min<int64_t>({16, J, std::max<int64_t>(1, (J + len - 1) / len)});
        q.order[i] = i;
        q.slots += g[i]->ncell * q.nchunk[i];
        q.cells += g[i]->ncell;
    }
    q.items = q.slots;
    auto cost = [&](int i) { return (g[i]->plan->J + q.nchunk[i] - 1) / q.nchunk[i]; };
    std::stable_sort(q.order, q.order + nseg, [&](int a, int b) { return cost(a) > cost(b); });
    return q;
}

template <int N>
hipError_t launch_queue(const fks_segment* const* g, int nseg, void* ws, hipStream_t st) {
    constexpr int NT = N * N / Cfg<N>::P;
    constexpr size_t HS = (size_t)(N / 2) * N * N;
    const QueuePlan qp = queue_plan(g, nseg);
    const fks_plan* p0 = g[0]->plan;
    char* base = (char*)ws;
    QueueArgs a{};
    a.fh = reinterpret_cast<cx<float>*>(base);
    const size_t part_off = align256((size_t)p0->fused_grid * HS * sizeof(cx<float>));
    a.part = reinterpret_cast<float*>(base + part_off);
    a.ctr = reinterpret_cast<int*>(base + part_off + align256((size_t)qp.slots * N * N * N * sizeof(float)));
    a.nseg = nseg;
    a.nitems = qp.items;
    a.ncell = qp.cells;
    int64_t item = 0, cell = 0;
    for (int k = 0; k < nseg; ++k) {
        const int i = qp.order[k];
        const fks_segment& s = *g[i];
        QSeg& q = a.seg[k];
        q.f = s.f;
        q.f_base = s.f_base ? s.f_base : s.f;
        q.q_out = s.q_out;
        q.f_out = s.f_out;
        q.tab = reinterpret_cast<const cx<float>*>(s.plan->d_tab32p);
        q.gc = s.plan->d_gc;
        q.guard = s.plan->d_guard;
        q.dt = s.dt_over_tau;
        q.item0 = item;
        q.part0 = item;   // one partial slot per item, in item order
        q.cell0 = cell;
        q.J = s.plan->J;
        q.nchunk = qp.nchunk[i];
        item += s.ncell * q.nchunk;
        cell += s.ncell;
    }
    k_zero_counter<<<1, 64, 0, st>>>(a.ctr);
    hipError_t e = hipGetLastError();
    if (e == hipSuccess) e = prof_mark(0, st);
    if (e != hipSuccess) return e;
    const int64_t grid = std::min<int64_t>(p0->fused_grid, qp.items);
    k_terms<N, 2><<<(unsigned)grid, NT, 0, st>>>(a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = prof_mark(1, st)) != hipSuccess) return e;
    k_finish_q<N><<<(unsigned)qp.cells, finish_threads<N>(), 0, st>>>(a);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return prof_mark(2, st);
}

}  // namespace

namespace {
// n = 48: the forward transform (multi-pass, into the half spectrum), the on-chip terms
// kernel with three workgroups per cell, then the FP64 fix and update, per chunk of at most
// kChunk48 cells.  Workspace per chunk: the complex n^3 work array of the forward passes,
// reused as the FP32 accumulator once the spectrum is built; the half spectrum; the
// workgroups' item counters.
constexpr int64_t kChunk48 = 512;
struct Ws48 {
    int64_t chunk;
    size_t fh, ctr, total;
};
inline Ws48 ws48(int64_t ncell) {
    constexpr size_t N3 = 48 * 48 * 48, H = 25 * 48 * 48;
    Ws48 w{};
    w.chunk = std::min<int64_t>(std::max<int64_t>(ncell, 1), kChunk48);
    w.fh = align256((size_t)w.chunk * N3 * sizeof(cx<float>));
    w.ctr = w.fh + align256((size_t)w.chunk * H * sizeof(cx<float>));
    w.total = w.ctr + 256;
    return w;
}

// Segments of n = 48 in one call: cells are taken in chunks of at most kChunk48, segments
// ordered by term count (longest first, so that the per-XCD queues end evenly); a chunk is
// a list of pieces (a segment's cell range).  Per chunk: the forward transform of every
// piece, one terms launch over all pieces, the fix and update of every piece.
hipError_t launch48(const fks_segment* const* g, int nseg, void* ws, hipStream_t st) {
    constexpr int64_t N3 = 48 * 48 * 48, H = 25 * 48 * 48;
    int64_t total = 0;
    for (int i = 0; i < nseg; ++i) total += g[i]->ncell;
    const Ws48 w = ws48(total);
    char* base = (char*)ws;
    cx<float>* work = reinterpret_cast<cx<float>*>(base);
    float* acc = reinterpret_cast<float*>(base);   // the work array once the spectrum is built
    cx<float>* fh = reinterpret_cast<cx<float>*>(base + w.fh);
    int* ctr = reinterpret_cast<int*>(base + w.ctr);
    std::vector<int> order(nseg);
    for (int i = 0; i < nseg; ++i) order[i] = i;
    std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return g[a]->plan->J > g[b]->plan->J; });
    struct Run {
        const fks_segment* s;
        int64_t c0, count;
    };
    int k = 0;
    int64_t next = 0;   // next cell of segment order[k]
    while (k < nseg) {
        std::vector<Run> runs;
        int64_t C = 0;
        while (k < nseg && C < w.chunk && (int)runs.size() < kMaxPieces48) {
            const fks_segment* s = g[order[k]];
            const int64_t take = std::min(s->ncell - next, w.chunk - C);
            runs.push_back(Run{s, next, take});
            C += take;
            next += take;
            if (next == s->ncell) {
                ++k;
                next = 0;
            }
        }
        Piece48 pc[kMaxPieces48];
        int64_t off = 0;
        hipError_t e = hipSuccess;
        for (size_t i = 0; i < runs.size() && e == hipSuccess; ++i) {
            const Run& r = runs[i];
            pc[i] = Piece48{reinterpret_cast<const cx<float>*>(r.s->plan->d_tab32p), off, r.s->plan->J};
            e = forward_f32_48(r.s->f + r.c0 * N3, work + off * N3, fh + off * H, (int)r.count, st);
            off += r.count;
        }
        if (e == hipSuccess) e = prof_mark(0, st);
        if (e == hipSuccess) e = terms48(fh, pc, (int)runs.size(), acc, C, ctr, g[0]->plan->fused_grid, st);
        if (e == hipSuccess) e = prof_mark(1, st);
        Fin48 fin[kMaxPieces48];
        off = 0;
        for (size_t i = 0; i < runs.size(); ++i) {
            const Run& r = runs[i];
            const fks_segment& s = *r.s;
            fin[i] = Fin48{s.f_base ? s.f_base : s.f, s.q_out, s.f_out, s.plan->d_gc, s.plan->d_guard,
                           s.dt_over_tau, off, r.c0};
            off += r.count;
        }
        if (e == hipSuccess) e = finish48(acc, fin, (int)runs.size(), C, st);
        if (e == hipSuccess) e = prof_mark(2, st);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
}  // namespace

int fused_queue_max_segments() { return kMaxQSeg; }

size_t fused_queue_workspace_bytes(const fks_segment* const* g, int nseg) {
    const int n = g[0]->plan->desc.n;
    if (n == 48) {
        int64_t total = 0;
        for (int i = 0; i < nseg; ++i) total += g[i]->ncell;
        return ws48(total).total;
    }
    const QueuePlan qp = queue_plan(g, nseg);
    const size_t HS = (size_t)(n / 2) * n * n;
    return align256((size_t)g[0]->plan->fused_grid * HS * sizeof(cx<float>)) +
           align256((size_t)qp.slots * n * n * n * sizeof(float)) + 256;
}

hipError_t collide_fused_queue(const fks_segment* const* g, int nseg, void* ws, size_t ws_bytes, hipStream_t st) {
    if (nseg < 1 || nseg > kMaxQSeg || ws_bytes < fused_queue_workspace_bytes(g, nseg)) return hipErrorInvalidValue;
    switch (g[0]->plan->desc.n) {
        case 48: return launch48(g, nseg, ws, st);
        case 8: return launch_queue<8>(g, nseg, ws, st);
        case 16: return launch_queue<16>(g, nseg, ws, st);
        case 24: return launch_queue<24>(g, nseg, ws, st);
        case 32: return launch_queue<32>(g, nseg, ws, st);
        default: return hipErrorInvalidValue;
    }
}

void profile_enable(bool on) {
    g_prof.on = on;
    g_prof.count = 0;
}

hipError_t profile_last(double* ms, int cap, int* count) {
    *count = 0;
    if (!g_prof.made || g_prof.count < 1) return hipSuccess;
    const int last = g_prof.count;   // 1: one kernel (one workgroup per cell), 2: terms + finish
    hipError_t e = hipEventSynchronize(g_prof.ev[last]);
    if (e != hipSuccess) return e;
    int n = 0;
    for (int i = 0; i < last && n < cap; ++i) {
        float t = 0.0f;
        if ((e = hipEventElapsedTime(&t, g_prof.ev[i], g_prof.ev[i + 1])) != hipSuccess) return e;
        ms[n++] = t;
    }
    *count = n;
    return hipSuccess;
}

bool fused_available(int n) { return n == 8 || n == 16 || n == 24 || n == 32 || n == 48; }

int fused_grid_size(int n, int device) {
    switch (n) {
        case 8: return grid_for<8>(device);
        case 16: return grid_for<16>(device);
        case 24: return grid_for<24>(device);
        case 32: return grid_for<32>(device);
        case 48: return terms48_grid(device);
        default: return 0;
    }
}


size_t fused_workspace_bytes(const fks_plan* p, int64_t ncell) {
    return p->desc.n == 48 ? ws48(ncell).total : ws_layout(p, ncell).total;
}

hipError_t collide_fused(const fks_plan* p, const fks_segment& s, void* ws, size_t ws_bytes, hipStream_t st) {
    if (ws_bytes < fused_workspace_bytes(p, s.ncell)) return hipErrorInvalidValue;
    switch (p->desc.n) {
        case 48: {
            const fks_segment* one = &s;
            return launch48(&one, 1, ws, st);
        }
        case 8: return launch<8>(p, s, ws, st);
        case 16: return launch<16>(p, s, ws, st);
        case 24: return launch<24>(p, s, ws, st);
        case 32: return launch<32>(p, s, ws, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fks
