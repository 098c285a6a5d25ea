// FP32 collision terms at n = 48, on chip, three workgroups per cell.
//
// One cell's complex 48^3 state (885 KB in FP32) does not fit one CU, so the inverse
// transform of every term is split by the residue of the output x modulo 3.  With
// x = 3m + r and kx = k1 + 16 k2 (k1 < 16, k2 < 3), exp(2 pi i kx x / 48) factors as
// exp(2 pi i k1 m / 16) w48^(r k1) w3^(r k2), so the x ≡ r part of
//   z(x, y, z) = sum_k Z(k) exp(2 pi i k.x / 48),   Z = (a_j + i b_j) fhat   (eq. ode)
// needs only the 16 combined planes
//   Y_r(k1, ky, kz) = w48^(r k1) sum_k2 w3^(r k2) Z(k1 + 16 k2, ky, kz),
// their z and y inverse transforms (48 points) and 16-point transforms over k1.  A
// workgroup owns one (cell, r): it reads the whole half spectrum of the term (tables
// and fhat, from L2), keeps its 16 x 48 x 48 slice on chip and adds Re z Im z to its
// third of Q+: two thirds of those accumulators stay in registers over the terms, the
// last third is read and written in the workspace every term (keeping all of them in
// registers, or none, spills more and ran slower).  No data
// moves between workgroups; the FP64 fix runs afterwards over the whole cell.
//
// Thread layouts (768 threads, 12 waves):
//   Z stage: combined pencil (k1, ky), registers over kz.  fhat is Hermitian and the
//     tables even, so the values at kz > 24 come from the loads of the mirror pencil
//     (-k1 mod 16, -ky).  Mirror pencils sit in lanes i and 15 - i of one 16-lane row:
//     each lane loads its own half (kz < 24, three kx), forms its own values and the
//     ones its mirror needs, M = w48^(-r k1) sum_k2 w3^(-r k2) t_k2 conj(f_k2), and a
//     row-mirror DPP move exchanges M.  The four self-mirrored pencils ((0,0), (8,0),
//     (0,24), (8,24)) keep their own M.
//   B stage: pencil (k1, z), registers over ky; the A -> B exchange goes through LDS in
//     two rounds (real parts, then imaginary parts: 147 KB each).
//   C stage: pencil (y, z), registers over k1, in three rounds of 16 y (98 KB each),
//     round rho the y = 3 yl + rho, which the y transform's 16-point group rho holds;
//     each round's pencil is transformed and accumulated at once.  The A -> B real
//     parts of each 16-point group of the z transform, and round 0 of B -> C, go out
//     as their group is formed.
// Work items (cell, r) come from one counter per XCD: workgroup b takes items of the
// cells c with c mod 8 = b mod 8 (blocks are dispatched to XCDs round-robin), so the
// three residues of a cell share fhat in one XCD's L2.
#include <hip/hip_runtime.h>

#include "fks_common.hpp"

namespace fks {
namespace {

constexpr int kN48 = 48;
constexpr int kThreads48 = 768;

struct W48Table {
    cx<float> w[48];
};
constexpr W48Table make_w48() {
    W48Table t{};
    for (int k = 0; k < 48; ++k) {
        const ct::sc s = ct::sincos2pi(k, 48);
        t.w[k] = cx<float>{float(s.c), float(s.s)};
    }
    return t;
}
__constant__ W48Table c_w48 = make_w48();   // exp(2 pi i k / 48)

// value held by lane (l & ~15) | (15 - (l & 15)) (row-mirror DPP move)
__device__ __forceinline__ float from_mirror_lane(float v) {
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x140, 0xf, 0xf, false));
}

__device__ __forceinline__ cx<float> cmul(cx<float> a, cx<float> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
__device__ __forceinline__ cx<float> cmul_conj_b(cx<float> a, cx<float> b) {   // a conj(b)
    return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
__device__ __forceinline__ cx<float> conjf(cx<float> a) { return {a.x, -a.y}; }

// Hides a value from loop-invariant code motion: per-thread offsets are recomputed next to
// their loads instead of being hoisted out of the term loop (72 spectrum addresses would
// not fit the registers).
template <typename V>
__device__ __forceinline__ V opaque48(V v) {
    asm volatile("" : "+v"(v));
    return v;
}

// 48-point transform (exp(+2 pi i n k / 48)): radix-3 decimation in frequency, then three
// in-place 16-point transforms, one at a time, so that the live set stays near the 48
// values; X[k] ends in x[slot48(k)] = x[16 (k mod 3) + k / 3]
template <typename Hook>
__device__ __forceinline__ void fft48_dif(cx<float> (&x)[48], Hook&& hook) {
    sfor<16>([&](auto nI) {
        constexpr int n1 = decltype(nI)::value;
        cx<float> u[3] = {x[n1], x[n1 + 16], x[n1 + 32]};
        butterfly<float, 3, 1>(u);
        x[n1] = u[0];
        x[n1 + 16] = twiddle<float, 1, 48, n1>(u[1]);
        x[n1 + 32] = twiddle<float, 1, 48, 2 * n1>(u[2]);
    });
    sfor<3>([&](auto qI) {
        constexpr int q = decltype(qI)::value;
        __builtin_amdgcn_sched_barrier(0);
        cx<float> s[16];
        sfor<16>([&](auto kI) { s[decltype(kI)::value] = x[16 * q + decltype(kI)::value]; });
        fft<float, 16, 1>(s);
        sfor<16>([&](auto kI) { x[16 * q + decltype(kI)::value] = s[decltype(kI)::value]; });
        hook(qI);   // slots 16 q .. 16 q + 15 (outputs k = 3 m + q) are final here
    });
    __builtin_amdgcn_sched_barrier(0);
}
__device__ __forceinline__ void fft48_dif(cx<float> (&x)[48]) {
    fft48_dif(x, [](auto) {});
}
constexpr int slot48(int k) { return 16 * (k % 3) + k / 3; }

struct Args48 {
    const cx<float>* fh;   // [C][25][48][48] (kz, kx, ky), scaled by n^-3, Nyquist planes zero
    float* acc;            // [C][48][48][48] Q+ (each residue writes its planes x = 3m + r)
    int64_t C;
    int* ctr;              // [8] item counters, zero at launch
    Piece48 pc[kMaxPieces48];   // cell ranges sharing a plan, in the order of the cells
    int npc;
};

// the piece of cell c: the last one starting at or before c (compile-time indices keep the
// argument table in scalar registers)
__device__ __forceinline__ Piece48 piece_of(const Args48& A, int64_t c) {
    Piece48 cur = A.pc[0];
    sfor<kMaxPieces48>([&](auto kI) {
        constexpr int k = decltype(kI)::value;
        if constexpr (k > 0) {
            if (k < A.npc && A.pc[k].cell0 <= c) cur = A.pc[k];
        }
    });
    return cur;
}

__global__ __launch_bounds__(kThreads48) void k_reset_counters(int* ctr) {
    if (threadIdx.x < 8) ctr[threadIdx.x] = 0;
}

__global__ __launch_bounds__(kThreads48) void k_terms48(Args48 A) {
    constexpr int N = kN48;
    constexpr int NN = N * N;
    constexpr int N3 = N * N * N;
    constexpr int H = (N / 2 + 1) * NN;   // spectrum slot stride
    constexpr int HT = (N / 2) * NN;      // table stride (planes kz < n/2, kz pairs adjacent)
    constexpr int RSA = N + 1;            // A -> B row stride (floats)
    constexpr int RSC = 17;               // B -> C row stride (complex)
    __shared__ float lds[16 * N * RSA];   // 150528 bytes
    __shared__ int s_item;
    cx<float>* const ldc = reinterpret_cast<cx<float>*>(lds);

    const int t = threadIdx.x;
    const int w = t >> 6, l = t & 63;
    // Z-stage pencil (k1, ky): pair index p = 32 w + 8 row + i' (i' < 8); lane i of a row
    // holds member 0 of pair i' = i, lane 15 - i member 1
    int k1, ky;
    bool self;
    {
        const int i = l & 15, h = i >> 3, ii = h ? 15 - i : i;
        const int p = w * 32 + (l >> 4) * 8 + ii;
        self = p >= 382;
        if (p < 336) {
            const int a = 1 + p / 48, b = p % 48;
            k1 = h ? 16 - a : a;
            ky = h ? (48 - b) % 48 : b;
        } else if (p < 382) {
            const int q = p - 336, b = 1 + q % 23;
            k1 = (q / 23) * 8;
            ky = h ? 48 - b : b;
        } else {
            k1 = h ? 8 : 0;
            ky = p == 382 ? 0 : 24;
        }
    }
    const int ub = t / N, uz = t % N;   // B stage (k1, z) and C stage (y within the round, z)
    const int xcd = blockIdx.x & 7;

    for (;;) {
        if (t == 0) s_item = atomicAdd(A.ctr + xcd, 1);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        const int64_t cell = xcd + 8 * (int64_t)(item / 3);
        if (cell >= A.C) break;
        const int r = item % 3;
        const cx<float> tw = c_w48.w[(r * k1) % 48];
        const cx<float> w3 = c_w48.w[16 * r], w3b = c_w48.w[(32 * r) % 48];
        const Piece48 pce = piece_of(A, cell);
        const char* const fhb = reinterpret_cast<const char*>(A.fh + cell * (int64_t)H);
        // Q+ of this third of the cell: node (3m + r, 3 ub + rho, uz), at byte offset
        // 4 (3m NN + rho N) + qo from the uniform base; rounds rho = 0, 1 accumulate in
        // registers, round 2 in place in the workspace
        char* const qb = reinterpret_cast<char*>(A.acc + cell * (int64_t)N3 + r * NN);
        float q0[2][16];   // rounds 0 and 1
        sfor<2>([&](auto rI) { sfor<16>([&](auto mI) { q0[decltype(rI)::value][decltype(mI)::value] = 0.0f; }); });

        for (int j = 0; j < pce.J; ++j) {
            const char* const tjb = reinterpret_cast<const char*>(pce.tab + (size_t)j * HT);
            const uint32_t ob = opaque48(uint32_t(k1 * N + ky) * 16u);
            cx<float> y[N];
            // ---- Z stage: combined products over kz ----
            // table and spectrum hold the planes kz = 2m, 2m + 1 side by side, so one 16-byte
            // load brings both: half the load instructions of 8-byte loads.  Pairs 0 and 1 are
            // loaded before the first products, pair 2 once pair 0's products are formed, and
            // from then on pair m + 1 once pair m's are (the other waves of the SIMD cover the
            // rest of the wait; two pairs ahead throughout spills)
            constexpr int NP = N / 4;   // kz pairs
            cx<float> tv[NP][3][2], fv[NP][3][2];
            auto load_pair = [&](auto mI) {
                constexpr int m = decltype(mI)::value;
                sfor<3>([&](auto cI) {
                    constexpr int c2 = decltype(cI)::value;
                    constexpr uint32_t zo = (m * NN + 16 * N * c2) * 16u;
                    const float4 a = *reinterpret_cast<const float4*>(tjb + (ob + zo));
                    const float4 b = *reinterpret_cast<const float4*>(fhb + (ob + zo));
                    tv[m][c2][0] = {a.x, a.y};
                    tv[m][c2][1] = {a.z, a.w};
                    fv[m][c2][0] = {b.x, b.y};
                    fv[m][c2][1] = {b.z, b.w};
                });
            };
            // pairs issued once pair m is done (m = -1: before the first)
            constexpr auto issued = [](int m) {
                const int u = m < 1 ? m + 3 : m + 2;
                return u < NP ? u : NP;
            };
            sfor<issued(-1)>([&](auto mI) { load_pair(mI); });
            sfor<N / 2>([&](auto kI) {
                constexpr int kz = decltype(kI)::value;
                constexpr int b = kz / 2, e = kz % 2;
                const cx<float> p0 = cmul(tv[b][0][e], fv[b][0][e]), p1 = cmul(tv[b][1][e], fv[b][1][e]),
                                p2 = cmul(tv[b][2][e], fv[b][2][e]);
                const cx<float> s = cadd(p0, cadd(cmul(w3, p1), cmul(w3b, p2)));
                y[kz] = cmul(tw, s);
                if constexpr (kz > 0) {
                    const cx<float> m0 = cmul_conj_b(tv[b][0][e], fv[b][0][e]), m1 = cmul_conj_b(tv[b][1][e], fv[b][1][e]),
                                    m2 = cmul_conj_b(tv[b][2][e], fv[b][2][e]);
                    const cx<float> sm = cadd(m0, cadd(cmul(conjf(w3), m1), cmul(conjf(w3b), m2)));
                    const cx<float> m = cmul(conjf(tw), sm);
                    const cx<float> mm = {from_mirror_lane(m.x), from_mirror_lane(m.y)};
                    y[N - kz] = self ? m : mm;
                }
                if constexpr (e == 1)
                    sfor<issued(kz / 2) - issued(kz / 2 - 1)>([&](auto qI) {
                        load_pair(std::integral_constant<int, issued(kz / 2 - 1) + decltype(qI)::value>{});
                    });
                __builtin_amdgcn_sched_barrier(0);
            });
            y[N / 2] = cx<float>{0.0f, 0.0f};
            // ---- A -> B: real parts, then imaginary parts ----
            __syncthreads();   // the previous C round has read the LDS
            float* const arow = lds + opaque48((k1 * N + ky) * RSA);
            // over kz (registers over z, z in slot48(z)); each 16-point group's real parts go
            // out as the group is formed (group q holds z = 3 k + q in slots 16 q + k)
            fft48_dif(y, [&](auto qI) {
                constexpr int q = decltype(qI)::value;
                __builtin_amdgcn_sched_barrier(0);
                sfor<16>([&](auto kI) {
                    constexpr int k = decltype(kI)::value;
                    arow[3 * k + q] = y[16 * q + k].x;
                });
                __builtin_amdgcn_sched_barrier(0);
            });
            __syncthreads();
            // LDS bases recomputed in each phase (opaque): hoisted out of the term loop, the
            // dozen bases that the paired LDS accesses need would stay live and spill
            cx<float> bv[N];
            const float* const brow = lds + opaque48(ub * N * RSA + uz);
            sfor<N>([&](auto kI) {
                constexpr int kk = decltype(kI)::value;
                bv[kk].x = brow[kk * RSA];
            });
            __syncthreads();
            sfor<N>([&](auto zI) { arow[decltype(zI)::value] = y[slot48(decltype(zI)::value)].y; });
            __syncthreads();
            const float* const brow2 = lds + opaque48(ub * N * RSA + uz);
            sfor<N>([&](auto kI) {
                constexpr int kk = decltype(kI)::value;
                bv[kk].y = brow2[kk * RSA];
            });
            // ---- B -> C in three rounds, round rho the 16 y = 3 yl + rho (slots 16 rho + yl);
            // x transform and accumulation per round ----
            __syncthreads();   // every thread has read its imaginary parts
            // over ky (registers over y, y in slot48(y)); round 0's writes go out as its group
            // of the transform is formed
            fft48_dif(bv, [&](auto qI) {
                if constexpr (decltype(qI)::value == 0) {
                    __builtin_amdgcn_sched_barrier(0);
                    cx<float>* const crow = ldc + opaque48(uz * RSC + ub);
                    sfor<16>([&](auto yI) {
                        constexpr int yl = decltype(yI)::value;
                        crow[yl * N * RSC] = bv[yl];
                    });
                    __builtin_amdgcn_sched_barrier(0);
                }
            });
            sfor<3>([&](auto rhoI) {
                constexpr int rho = decltype(rhoI)::value;
                if constexpr (rho > 0) {
                    __syncthreads();
                    cx<float>* const crow = ldc + opaque48(uz * RSC + ub);
                    sfor<16>([&](auto yI) {
                        constexpr int yl = decltype(yI)::value;
                        crow[yl * N * RSC] = bv[16 * rho + yl];
                    });
                }
                // this round's accumulators, loaded once the round's B values have left the
                // registers; their latency overlaps the exchange and the x transform
                float prev[16];
                const uint32_t qo = opaque48(uint32_t(3 * ub * N + uz) * 4u);
                sfor<16>([&](auto mI) { prev[decltype(mI)::value] = 0.0f; });
                if (rho > 1 && j > 0) {
                    sfor<16>([&](auto mI) {
                        constexpr int m = decltype(mI)::value;
                        constexpr uint32_t mo = (3 * m * NN + rho * N) * 4u;
                        prev[m] = *reinterpret_cast<const float*>(qb + (qo + mo));
                    });
                }
                __syncthreads();
                cx<float> xc[16];
                const cx<float>* const xrow = ldc + opaque48((ub * N + uz) * RSC);
                sfor<16>([&](auto kI) {
                    constexpr int kk = decltype(kI)::value;
                    xc[kk] = xrow[kk];
                });
                fft<float, 16, 1>(xc);   // over k1: x = 3m + r
                sfor<16>([&](auto mI) {
                    constexpr int m = decltype(mI)::value;
                    constexpr uint32_t mo = (3 * m * NN + rho * N) * 4u;
                    if constexpr (rho < 2) q0[rho][m] = fmaf(xc[m].x, xc[m].y, q0[rho][m]);
                    else *reinterpret_cast<float*>(qb + (qo + mo)) = fmaf(xc[m].x, xc[m].y, prev[m]);
                });
            });
        }
        {
            const uint32_t qo = uint32_t(3 * ub * N + uz) * 4u;
            sfor<2>([&](auto rI) {
                constexpr int rho = decltype(rI)::value;
                sfor<16>([&](auto mI) {
                    constexpr int m = decltype(mI)::value;
                    *reinterpret_cast<float*>(qb + (qo + uint32_t(3 * m * NN + rho * N) * 4u)) = q0[rho][m];
                });
            });
        }
    }
}

// FP64 fix and update of every cell of a chunk (all pieces in one launch): Q+ (FP32,
// the terms kernel's output) -> moments in FP64 -> lambda = G^{-1} C Q -> Q_c = Q - C^T lambda
// -> q_out and/or f_out = f_base + dt/tau Q_c (eqs. minim1, f_coll).  One workgroup of 768
// threads per cell; thread t owns the x pencils of (y, z) = (t / 48 + 16 i, t mod 48),
// i < 3 (coalesced over z); Q is read twice (moments, then the update).
struct FinArgs48 {
    const float* acc;      // [C][48^3]
    int64_t C;
    Fin48 pc[kMaxPieces48];
    int npc;
};

__device__ __forceinline__ Fin48 fin_piece_of(const FinArgs48& A, int64_t c) {
    Fin48 cur = A.pc[0];
    sfor<kMaxPieces48>([&](auto kI) {
        constexpr int k = decltype(kI)::value;
        if constexpr (k > 0) {
            if (k < A.npc && A.pc[k].cell0 <= c) cur = A.pc[k];
        }
    });
    return cur;
}

__global__ __launch_bounds__(kThreads48) void k_finish48(FinArgs48 A) {
    constexpr int N = kN48, NN = N * N, N3 = N * N * N;
    __shared__ double red[5 * (kThreads48 / 64)];
    const int t = threadIdx.x;
    const int64_t cell = blockIdx.x;
    const Fin48 pc = fin_piece_of(A, cell);
    const int64_t lc = cell - pc.cell0;                 // cell within the piece
    const float* const q = A.acc + cell * (int64_t)N3;
    const double h = pc.gc->dv / pc.gc->T;
    const int yb = t / N, z = t % N;
    const double uz = -1.0 + z * h;
    double m[5] = {0, 0, 0, 0, 0};
    for (int i = 0; i < 3; ++i) {
        const int y = yb + 16 * i;
        const double uy = -1.0 + y * h;
        const double ryz = fma(uy, uy, uz * uz);
        const float* const pq = q + y * N + z;
#pragma unroll 8
        for (int x = 0; x < N; ++x) {
            const double ux = -1.0 + x * h;
            const double v = (double)pq[x * NN];
            m[0] += v;
            m[1] = fma(v, ux, m[1]);
            m[2] = fma(v, uy, m[2]);
            m[3] = fma(v, uz, m[3]);
            m[4] = fma(v, fma(ux, ux, ryz), m[4]);
        }
    }
    block_sum5<kThreads48>(m, red);
    if (pc.guard && t == 0 && !isfinite(m[0] + m[1] + m[2] + m[3] + m[4]))
        atomicMin(pc.guard, (unsigned long long)(pc.c0 + lc));
    double lam[5];
    solve5(*pc.gc, m, lam);
    const int64_t base = (pc.c0 + lc) * (int64_t)N3;
    for (int i = 0; i < 3; ++i) {
        const int y = yb + 16 * i;
        const double uy = -1.0 + y * h;
        const double lyz = fma(lam[4], fma(uy, uy, uz * uz), fma(lam[2], uy, fma(lam[3], uz, lam[0])));
        const int off = y * N + z;
#pragma unroll 8
        for (int x = 0; x < N; ++x) {
            const double ux = -1.0 + x * h;
            const double v = (double)q[off + x * NN] - fma(lam[4], ux * ux, fma(lam[1], ux, lyz));
            const int64_t o = base + off + x * NN;
            if (pc.q_out) __builtin_nontemporal_store(v, pc.q_out + o);
            if (pc.f_out) __builtin_nontemporal_store(fma(pc.dt, v, __builtin_nontemporal_load(pc.f_base + o)), pc.f_out + o);
        }
    }
}

}  // namespace

hipError_t finish48(const float* acc, const Fin48* pieces, int npieces, int64_t ncell, hipStream_t st) {
    if (npieces < 1 || npieces > kMaxPieces48) return hipErrorInvalidValue;
    FinArgs48 a{};
    a.acc = acc;
    a.C = ncell;
    a.npc = npieces;
    for (int i = 0; i < npieces; ++i) a.pc[i] = pieces[i];
    k_finish48<<<(unsigned)ncell, kThreads48, 0, st>>>(a);
    return hipGetLastError();
}

int terms48_grid(int device) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0)
        cus = 256;
    int per = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_terms48, kThreads48, 0) != hipSuccess || per <= 0)
        per = 1;
    return std::max(8, (cus * per / 8) * 8);
}

hipError_t terms48(const cx<float>* fh, const Piece48* pieces, int npieces, float* acc, int64_t ncell, int* ctr,
                   int grid, hipStream_t st) {
    if (npieces < 1 || npieces > kMaxPieces48) return hipErrorInvalidValue;
    k_reset_counters<<<1, 64, 0, st>>>(ctr);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    Args48 a{};
    a.fh = fh;
    a.acc = acc;
    a.C = ncell;
    a.ctr = ctr;
    a.npc = npieces;
    for (int i = 0; i < npieces; ++i) a.pc[i] = pieces[i];
    k_terms48<<<(unsigned)grid, kThreads48, 0, st>>>(a);
    return hipGetLastError();
}

}  // namespace fks
