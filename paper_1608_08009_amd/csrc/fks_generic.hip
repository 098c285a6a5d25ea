// Multi-pass collision path (FP64 "plain" path, and FP32 for sizes without a
// fused kernel).  Every 3D transform is three pencil passes through a device
// workspace; the conservation projection and update run in FP64.
//
// Per chunk of cells:
//   forward:  x-pass, y-pass, z-pass -> fhat (half spectrum kz in [0, n/2],
//             scaled by n^-3, Nyquist planes zeroed)                 (eq. FC)
//   per term j (M*K gain terms, then the loss term):
//             fused z- and y-pass per (cell, kx) plane with Z = (a_j + i b_j) fhat
//             on input, then the x-pass with acc += Re(z) Im(z) on output
//             (eq. ode, fast form)
//   finish:   FP64 moments of acc, lambda = G^{-1} C acc, Q_c = acc - C^T lambda,
//             outputs q_out = Q_c and/or f_out = f_base + dt/tau Q_c (eqs. minim1, f_coll)
// Plans with FKS_FLAG_DEALIAS take the zero-padded variant described below.
#include <hip/hip_runtime.h>

#include "fks_common.hpp"

namespace fks {

bool generic_multi_terms(const fks_plan* p) {
    return !(p->desc.precision == FKS_PREC_F64 && p->desc.n >= 48) && !(p->desc.flags & FKS_FLAG_DEALIAS);
}

namespace {

constexpr int kChunk = 512;          // cells per pass batch
constexpr int kChunkOneTerm = 128;   // cells per pass batch where each launch takes one term (n >= 32)
constexpr int kTermsPerLaunch = 4;   // consecutive terms per launch of the per-term kernels

// consecutive terms per launch of the per-term kernels: the measured choice of
// fks_autotune, else the default (one where the loop does not fit the registers)
inline int terms_per_launch(const fks_plan* p, int64_t ncell) {
    if (!generic_multi_terms(p)) return 1;
    const Schedule sc = schedule_for(p, ncell);
    return sc.terms > 0 ? sc.terms : kTermsPerLaunch;
}

// cells per pass batch: the measured choice of fks_autotune, else the default.  With four
// terms per launch, 512-cell batches were the fastest measured (4096 cells of 32^3 in FP64:
// 61.6 ms; 1024 cells of 48^3 in FP32: 29.7 ms).  Where each launch takes one term (the
// de-aliased variant, FP64 at n = 48) smaller batches keep more of the work arrays in the
// caches (4096 cells of 32^3 in FP64, one term per launch: 64 ms with 128 cells against
// 76 ms with 512).
inline int chunk_cells(const fks_plan* p, int64_t ncell) {
    const Schedule sc = schedule_for(p, ncell);
    if (sc.chunk > 0) return sc.chunk;
    // the n = 48 kernel's three workgroups per cell need several cells per resident workgroup
    if ((p->desc.flags & FKS_FLAG_DEALIAS) && p->d_tab48p) return kChunk;
    if ((p->desc.flags & FKS_FLAG_DEALIAS) || (!generic_multi_terms(p) && p->desc.n >= 32)) return kChunkOneTerm;
    return kChunk;
}

template <typename T>
struct Tab;
template <>
struct Tab<double> {
    static const cx<double>* get(const fks_plan* p) { return reinterpret_cast<const cx<double>*>(p->d_tab64); }
};
template <>
struct Tab<float> {
    static const cx<float>* get(const fks_plan* p) { return reinterpret_cast<const cx<float>*>(p->d_tab32); }
};

template <typename T, int N>
__global__ __launch_bounds__(128) void g_fwd_x(const double* __restrict__ f, cx<T>* __restrict__ work, int C) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= C * N * N) return;
    const int z = t % N, y = (t / N) % N, c = t / (N * N);
    const double* src = f + (size_t)c * N * N * N + y * N + z;
    cx<T> v[N];
    sfor<N>([&](auto I) {
        constexpr int x = decltype(I)::value;
        v[x] = cx<T>{T(src[x * N * N]), T(0)};
    });
    fft<T, N, -1>(v);
    cx<T>* dst = work + (size_t)c * N * N * N + y * N + z;
    sfor<N>([&](auto I) {
        constexpr int k = decltype(I)::value;
        dst[k * N * N] = v[k];
    });
}

// in-place transform along y for pencils (c, kx, z); SIGN -1 forward, +1 inverse
template <typename T, int N, int SIGN>
__global__ __launch_bounds__(128) void g_pass_y(cx<T>* __restrict__ work, int C) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= C * N * N) return;
    const int z = t % N, kx = (t / N) % N, c = t / (N * N);
    cx<T>* p = work + (size_t)c * N * N * N + kx * N * N + z;
    cx<T> v[N];
    sfor<N>([&](auto I) {
        constexpr int y = decltype(I)::value;
        v[y] = p[y * N];
    });
    fft<T, N, SIGN>(v);
    sfor<N>([&](auto I) {
        constexpr int y = decltype(I)::value;
        p[y * N] = v[y];
    });
}

// PAIRS: the planes kz < n/2 in the kz-pair layout of the fused kernels, element (kz, kx, ky)
// at ((kz/2) n^2 + kx n + ky) 2 + kz % 2; plane n/2 stays at n/2 n^2 + kx n + ky
template <typename T, int N, bool PAIRS = false>
__global__ __launch_bounds__(128) void g_fwd_z(const cx<T>* __restrict__ work, cx<T>* __restrict__ fh, int C) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= C * N * N) return;
    const int ky = t % N, kx = (t / N) % N, c = t / (N * N);
    const cx<T>* p = work + (size_t)c * N * N * N + (kx * N + ky) * N;
    cx<T> v[N];
    sfor<N>([&](auto I) {
        constexpr int z = decltype(I)::value;
        v[z] = p[z];
    });
    fft<T, N, -1>(v);
    const T s = T(1.0 / ((double)N * N * N));
    const bool nyq = (kx == N / 2) || (ky == N / 2);
    constexpr int H = (N / 2 + 1) * N * N;
    cx<T>* o = fh + (size_t)c * H + kx * N + ky;
    sfor<N / 2 + 1>([&](auto I) {
        constexpr int kz = decltype(I)::value;
        cx<T> r = (nyq || kz == N / 2) ? cx<T>{T(0), T(0)} : cx<T>{v[kz].x * s, v[kz].y * s};
        if constexpr (PAIRS && kz < N / 2)
            fh[(size_t)c * H + ((kz / 2) * N * N + kx * N + ky) * 2 + kz % 2] = r;
        else
            o[kz * N * N] = r;
    });
}

// z and y inverse passes of one term fused, one (cell, kx) plane per group of n
// threads: thread ky computes Z = (a_j + i b_j) fhat over kz and its inverse
// transform over z; the plane goes through LDS (real parts, then imaginary parts,
// which halves the LDS per plane); thread z then transforms over y and writes
// work[c][kx][y][z] with consecutive lanes on consecutive z.
template <int N>
constexpr int zy_planes() { return N <= 32 ? 128 / N : 1; }

template <typename T, int N>
__device__ __forceinline__ void plane_sync() {
    if constexpr (64 % N == 0) {   // a plane's n threads lie in one wave
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// hides a pointer from loop-invariant code motion (the loads through it stay in the loop)
template <typename P>
__device__ __forceinline__ P hide(P p) {
    asm volatile("" : "+v"(p));
    return p;
}

// several terms per launch only where the loop state fits the registers (FP64 at n = 48
// already uses all 256 VGPRs for the transform)
template <typename T, int N>
constexpr bool multi_term_ok() { return !(sizeof(T) == 8 && N >= 48); }

template <typename T, int N, bool MT>
__global__ __launch_bounds__(zy_planes<N>() * N) void g_inv_zy(const cx<T>* __restrict__ fh,
                                                               const cx<T>* __restrict__ tab0,
                                                               cx<T>* __restrict__ work0, int C, int nt,
                                                               int64_t work_stride) {
    constexpr int PP = zy_planes<N>();
    constexpr int RS = N + 1;
    __shared__ T lds[PP * N * RS];
    const int pl = threadIdx.x / N, i = threadIdx.x % N;
    const int64_t plane = (int64_t)blockIdx.x * PP + pl;   // c * N + kx
    const bool live = plane < (int64_t)C * N;
    const int kx = (int)(plane % N);
    const int64_t c = live ? plane / N : 0;
    const int ky = i;
    const int mx = (N - kx) % N, my = (N - ky) % N;
    constexpr int H = (N / 2 + 1) * N * N;
    const cx<T>* const g0 = fh + c * H;
    const int nterm = MT ? nt : 1;
#pragma nounroll
    for (int t = 0; t < nterm; ++t) {   // nt consecutive terms, one work array each
    const cx<T>* const tab = tab0 + (size_t)t * H;
    cx<T>* const work = work0 + t * work_stride;
    // For n > 16, fhat is reloaded and the offsets recomputed every term (cache hits, a few
    // integer ops) rather than hoisted out of the loop into registers, which would cost the
    // kernel its occupancy; for n <= 16 the registers are there and the hoisting pays
    // (8192 cells of 16^3 in FP64: 12.1 -> 7.8 ms)
    constexpr bool keep = N <= 16;
    const cx<T>* const g = keep ? g0 : hide(g0);
    const int kxh = keep ? kx : hide(kx), kyh = keep ? ky : hide(ky);
    const int mxh = keep ? mx : hide(mx), myh = keep ? my : hide(my);
    cx<T> v[N];
    sfor<N>([&](auto I) {
        constexpr int kz = decltype(I)::value;
        cx<T> a, b;
        if constexpr (kz <= N / 2) {
            const int h = (kz * N + kxh) * N + kyh;
            a = tab[h];
            b = g[h];
        } else {
            const int h = ((N - kz) * N + mxh) * N + myh;   // fhat(-k) = conj fhat(k); tables even in k
            a = tab[h];
            b = g[h];
            b.y = -b.y;
        }
        v[kz] = cx<T>{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
    });
    fft<T, N, 1>(v);   // over kz: row ky = i, registers over z
    T* const blk = lds + pl * N * RS;
    cx<T> u[N];
    sfor<N>([&](auto I) { blk[i * RS + decltype(I)::value] = v[decltype(I)::value].x; });
    plane_sync<T, N>();
    sfor<N>([&](auto I) { u[decltype(I)::value].x = blk[decltype(I)::value * RS + i]; });
    plane_sync<T, N>();
    sfor<N>([&](auto I) { blk[i * RS + decltype(I)::value] = v[decltype(I)::value].y; });
    plane_sync<T, N>();
    sfor<N>([&](auto I) { u[decltype(I)::value].y = blk[decltype(I)::value * RS + i]; });
    fft<T, N, 1>(u);   // over ky: column z = i, registers over y
    if (live) {
        cx<T>* o = work + (c * N + kx) * N * N + i;
        sfor<N>([&](auto I) {
            constexpr int y = decltype(I)::value;
            o[y * N] = u[y];
        });
    }
    plane_sync<T, N>();   // the next term reuses the LDS block
    }
}

template <typename T, int N, bool MT>
__global__ __launch_bounds__(128) void g_inv_x(const cx<T>* __restrict__ work0, T* __restrict__ acc, int C,
                                               int first0, int nt, int64_t work_stride) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= C * N * N) return;
    const int z = t % N, y = (t / N) % N, c = t / (N * N);
    // nt consecutive terms: the accumulator lines stay in the caches between them
    const int nterm = MT ? nt : 1;
#pragma nounroll
    for (int term = 0; term < nterm; ++term) {
    const int first = first0 && term == 0;
    const cx<T>* p = hide(work0 + term * work_stride + (size_t)c * N * N * N + y * N + z);
    cx<T> v[N];
    sfor<N>([&](auto I) {
        constexpr int k = decltype(I)::value;
        v[k] = p[k * N * N];
    });
    fft<T, N, 1>(v);
    T* q = hide(acc + (size_t)c * N * N * N + y * N + z);
    if (first) {
        sfor<N>([&](auto I) {
            constexpr int x = decltype(I)::value;
            q[x * N * N] = v[x].x * v[x].y;
        });
    } else {
        // Accumulator read-modify-write.  The first-term test stays outside: a load under a
        // per-element condition is not speculated, and each one then waited for the memory
        // before the next was issued (48 round trips per thread at n = 48).  FP32 issues
        // every load before the first store; FP64 goes in fenced groups of x, since loading
        // every accumulator at once costs that kernel half its occupancy.
        constexpr int G = (sizeof(T) == 4 || N % 8 != 0) ? N : 8;
        sfor<N / G>([&](auto gI) {
            constexpr int g0 = decltype(gI)::value * G;
            T prod[G];
            sfor<G>([&](auto I) { prod[decltype(I)::value] = q[(g0 + decltype(I)::value) * N * N]; });
            sfor<G>([&](auto I) {
                constexpr int x = g0 + decltype(I)::value;
                q[x * N * N] = prod[decltype(I)::value] + v[x].x * v[x].y;
            });
            __builtin_amdgcn_sched_barrier(0);
        });
    }
    }
}

template <typename T, int N>
__global__ __launch_bounds__(256) void g_finish(const T* __restrict__ acc, const double* f,
                                                double* __restrict__ q_out, double* f_out, double dt,
                                                GridConst gc, unsigned long long* guard, int64_t c0) {
    __shared__ double red[5 * 4];
    __shared__ double lam_s[5];
    const int c = blockIdx.x;
    constexpr int NN = N * N * N;
    const T* q = acc + (size_t)c * NN;
    double m[5] = {0, 0, 0, 0, 0};
    for (int i = threadIdx.x; i < NN; i += 256) {
        const int z = i % N, y = (i / N) % N, x = i / (N * N);
        const Basis b = basis_at(gc, x, y, z);
        const double qv = (double)q[i];
#pragma unroll
        for (int a = 0; a < 5; ++a) m[a] = fma(qv, b.p[a], m[a]);
    }
    block_sum5<256>(m, red);
    if (threadIdx.x == 0) {
        if (guard && !isfinite(m[0] + m[1] + m[2] + m[3] + m[4])) atomicMin(guard, (unsigned long long)(c0 + c));
        double lam[5];
        solve5(gc, m, lam);
        for (int a = 0; a < 5; ++a) lam_s[a] = lam[a];
    }
    __syncthreads();
    double lam[5];
#pragma unroll
    for (int a = 0; a < 5; ++a) lam[a] = lam_s[a];
    const size_t base = (size_t)c * NN;
    for (int i = threadIdx.x; i < NN; i += 256) {
        const int z = i % N, y = (i / N) % N, x = i / (N * N);
        const double qc = (double)q[i] - correction(lam, basis_at(gc, x, y, z));
        if (q_out) q_out[base + i] = qc;
        if (f_out) f_out[base + i] = fma(dt, qc, f[base + i]);
    }
}

// Spectrum output pass: z transform of the y-passed work array, then
// xhat[c][kx][ky][kz] = (-1)^(kx+ky+kz) n^-3 DFT (eq. FC with v_j = -T + j dv:
// exp(-i kappa k.v_j) = (-1)^k exp(-2 pi i k j / n)), kz in [0, n/2], FP64.
template <int N>
__global__ __launch_bounds__(128) void g_spec_z(const cx<double>* __restrict__ work, double* __restrict__ xhat,
                                                int C, int zero_nyquist) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= C * N * N) return;
    const int ky = t % N, kx = (t / N) % N, c = t / (N * N);
    const cx<double>* p = work + (size_t)c * N * N * N + (kx * N + ky) * N;
    cx<double> v[N];
    sfor<N>([&](auto I) {
        constexpr int z = decltype(I)::value;
        v[z] = p[z];
    });
    fft<double, N, -1>(v);
    constexpr int HZ = N / 2 + 1;
    const double s = ((kx + ky) & 1 ? -1.0 : 1.0) / ((double)N * N * N);
    const bool nyq_xy = zero_nyquist && (kx == N / 2 || ky == N / 2);
    double* o = xhat + 2 * ((size_t)c * N * N * HZ + (size_t)(kx * N + ky) * HZ);
    sfor<HZ>([&](auto I) {
        constexpr int kz = decltype(I)::value;
        const double sk = (nyq_xy || (zero_nyquist && kz == N / 2)) ? 0.0 : ((kz & 1) ? -s : s);
        o[2 * kz] = v[kz].x * sk;
        o[2 * kz + 1] = v[kz].y * sk;
    });
}

template <int N>
hipError_t run_spectrum(const double* x, double* xhat, int64_t ncell, int zero_nyquist, void* ws, size_t ws_bytes,
                        hipStream_t st) {
    constexpr size_t NN = (size_t)N * N * N;
    const int64_t fit = (int64_t)(ws_bytes / (NN * sizeof(cx<double>)));
    const int chunk = (int)std::min<int64_t>(std::min<int64_t>(ncell, kChunk), fit);
    if (chunk < 1) return hipErrorInvalidValue;
    cx<double>* work = (cx<double>*)ws;
    const int bs = 128;
    for (int64_t c0 = 0; c0 < ncell; c0 += chunk) {
        const int C = (int)std::min<int64_t>(chunk, ncell - c0);
        const unsigned grid = (unsigned)((C * N * N + bs - 1) / bs);
        g_fwd_x<double, N><<<grid, bs, 0, st>>>(x + c0 * (int64_t)NN, work, C);
        g_pass_y<double, N, -1><<<grid, bs, 0, st>>>(work, C);
        g_spec_z<N><<<grid, bs, 0, st>>>(work, xhat + 2 * c0 * (int64_t)(N * N * (N / 2 + 1)), C, zero_nyquist);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ---------------------------------------------------------------------------
// De-aliased variant (zero-padded transforms).  The products a_j b_j and
// f_N F^{-1}(L fhat) are sampled on a grid of NP = 3n/2 points per axis of the
// same box, where no frequency of a product of two band-limited factors
// (|k_i| < n/2) folds back into the band; the band coefficients of the summed
// products then hold exactly the pairs l + m = k.  Layouts per cell (complex
// unless noted; k = n-grid wavenumber index in FFT order, primes = NP grid):
//   fh [kz <= n/2][kx][ky]  ->  W2 [kx][y'][z'] (z and y fused)  ->  acc [x'][y'][z'] (real)
//   acc -> W2 [kx][y'][z'] -> W1 [kx][ky][z'] -> W2 [kx][ky][z] (n^3) -> q [x][y][z] (real)
// ---------------------------------------------------------------------------

// index of n-grid wavenumber index k (k != n/2) in the NP-grid FFT order
template <int N, int NP>
constexpr int pad_pos(int k) { return k < N / 2 ? k : k - N + NP; }

// per term, x: zero-pad kx to NP, inverse transform, acc (+)= Re(z) Im(z) on the NP grid
template <typename T, int N, int NP>
__global__ __launch_bounds__(128) void d_pad_x(const cx<T>* __restrict__ w2, T* __restrict__ acc, int C, int first) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= C * NP * NP) return;
    const int zp = t % NP, yp = (t / NP) % NP, c = t / (NP * NP);
    const cx<T>* in = w2 + (size_t)c * N * NP * NP + yp * NP + zp;
    cx<T> v[NP];
    sfor<NP>([&](auto I) { v[decltype(I)::value] = cx<T>{T(0), T(0)}; });
    sfor<N>([&](auto I) {
        constexpr int kx = decltype(I)::value;
        if constexpr (kx != N / 2) v[pad_pos<N, NP>(kx)] = in[kx * NP * NP];
    });
    fft<T, NP, 1>(v);
    T* q = acc + (size_t)c * NP * NP * NP + yp * NP + zp;
    if (first) {
        sfor<NP>([&](auto I) {
            constexpr int x = decltype(I)::value;
            q[x * NP * NP] = v[x].x * v[x].y;
        });
    } else {
        // accumulator read-modify-write as in g_inv_x: unconditional loads, one group in FP32,
        // fenced groups in FP64
        constexpr int G = sizeof(T) == 4 ? NP : (NP % 8 == 0) ? 8 : (NP % 6 == 0 ? 6 : NP);
        sfor<NP / G>([&](auto gI) {
            constexpr int g0 = decltype(gI)::value * G;
            T prod[G];
            sfor<G>([&](auto I) { prod[decltype(I)::value] = q[(g0 + decltype(I)::value) * NP * NP]; });
            sfor<G>([&](auto I) {
                constexpr int x = g0 + decltype(I)::value;
                q[x * NP * NP] = prod[decltype(I)::value] + v[x].x * v[x].y;
            });
            __builtin_amdgcn_sched_barrier(0);
        });
    }
}

// per term, z and y fused: one wave per (cell, kx) plane.  Lanes ky < n compute Z over kz,
// zero-padded to NP, and transform over z'; the plane goes through LDS (real parts, then
// imaginary parts); lanes z' < NP then zero-pad ky, transform over y' and write
// W2[c][kx][y'][z'] with consecutive lanes on consecutive z'.
template <typename T, int N, int NP>
__global__ __launch_bounds__(64) void d_term_zy(const cx<T>* __restrict__ fh, const cx<T>* __restrict__ tab,
                                                cx<T>* __restrict__ w2, int C) {
    static_assert(NP <= 64 && N <= NP, "one wave per plane");
    constexpr int RS = NP + 1;
    __shared__ T lds[N * RS];
    const int i = threadIdx.x;
    const int64_t plane = blockIdx.x;   // c * N + kx
    const int kx = (int)(plane % N);
    const int64_t c = plane / N;
    constexpr int H = (N / 2 + 1) * N * N;
    cx<T> v[NP];
    if (i < N) {
        const int ky = i, mx = (N - kx) % N, my = (N - ky) % N;
        const cx<T>* g = fh + c * H;
        sfor<NP>([&](auto I) { v[decltype(I)::value] = cx<T>{T(0), T(0)}; });
        sfor<N>([&](auto I) {
            constexpr int kz = decltype(I)::value;
            if constexpr (kz != N / 2) {
                cx<T> a, b;
                if constexpr (kz < N / 2) {
                    const int h = (kz * N + kx) * N + ky;
                    a = tab[h];
                    b = g[h];
                } else {
                    const int h = ((N - kz) * N + mx) * N + my;   // fhat(-k) = conj fhat(k); tables even
                    a = tab[h];
                    b = g[h];
                    b.y = -b.y;
                }
                v[pad_pos<N, NP>(kz)] = cx<T>{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
            }
        });
        fft<T, NP, 1>(v);   // over z': row ky = i
        sfor<NP>([&](auto I) { lds[i * RS + decltype(I)::value] = v[decltype(I)::value].x; });
    }
    auto wsync = [] {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    };
    wsync();
    cx<T> u[NP];
    sfor<NP>([&](auto I) { u[decltype(I)::value] = cx<T>{T(0), T(0)}; });
    if (i < NP) {
        sfor<N>([&](auto I) {
            constexpr int ky = decltype(I)::value;
            if constexpr (ky != N / 2) u[pad_pos<N, NP>(ky)].x = lds[ky * RS + i];
        });
    }
    wsync();
    if (i < N) sfor<NP>([&](auto I) { lds[i * RS + decltype(I)::value] = v[decltype(I)::value].y; });
    wsync();
    if (i < NP) {
        sfor<N>([&](auto I) {
            constexpr int ky = decltype(I)::value;
            if constexpr (ky != N / 2) u[pad_pos<N, NP>(ky)].y = lds[ky * RS + i];
        });
        fft<T, NP, 1>(u);   // over y': column z' = i
        cx<T>* o = w2 + (c * N + kx) * NP * NP + i;
        sfor<NP>([&](auto I) {
            constexpr int y = decltype(I)::value;
            o[y * NP] = u[y];
        });
    }
}

// after the terms, x: forward transform of the real products over x', keep the band in kx
template <typename T, int N, int NP>
__global__ __launch_bounds__(128) void d_trunc_x(const T* __restrict__ acc, cx<T>* __restrict__ w2, int C) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= C * NP * NP) return;
    const int zp = t % NP, yp = (t / NP) % NP, c = t / (NP * NP);
    const T* in = acc + (size_t)c * NP * NP * NP + yp * NP + zp;
    cx<T> v[NP];
    sfor<NP>([&](auto I) {
        constexpr int x = decltype(I)::value;
        v[x] = cx<T>{in[x * NP * NP], T(0)};
    });
    fft<T, NP, -1>(v);
    cx<T>* o = w2 + (size_t)c * N * NP * NP + yp * NP + zp;
    sfor<N>([&](auto I) {
        constexpr int kx = decltype(I)::value;
        if constexpr (kx == N / 2) o[kx * NP * NP] = cx<T>{T(0), T(0)};
        else o[kx * NP * NP] = v[pad_pos<N, NP>(kx)];
    });
}

// y: forward transform over y', keep the band in ky
template <typename T, int N, int NP>
__global__ __launch_bounds__(128) void d_trunc_y(const cx<T>* __restrict__ w2, cx<T>* __restrict__ w1, int C) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= C * N * NP) return;
    const int zp = t % NP, kx = (t / NP) % N, c = t / (N * NP);
    const cx<T>* in = w2 + ((size_t)c * N + kx) * NP * NP + zp;
    cx<T> v[NP];
    sfor<NP>([&](auto I) {
        constexpr int y = decltype(I)::value;
        v[y] = in[y * NP];
    });
    fft<T, NP, -1>(v);
    cx<T>* o = w1 + ((size_t)c * N + kx) * N * NP + zp;
    sfor<N>([&](auto I) {
        constexpr int ky = decltype(I)::value;
        if constexpr (ky == N / 2) o[ky * NP] = cx<T>{T(0), T(0)};
        else o[ky * NP] = v[pad_pos<N, NP>(ky)];
    });
}

// z: forward transform over z', keep the band (Nyquist planes zero), scale NP^-3, then the
// inverse n-point transform over kz -> W2 [kx][ky][z]
template <typename T, int N, int NP>
__global__ __launch_bounds__(128) void d_trunc_z_inv(const cx<T>* __restrict__ w1, cx<T>* __restrict__ w2, int C) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= C * N * N) return;
    const int ky = t % N, kx = (t / N) % N, c = t / (N * N);
    const cx<T>* in = w1 + ((size_t)c * N * N + kx * N + ky) * NP;
    cx<T> v[NP];
    sfor<NP>([&](auto I) {
        constexpr int z = decltype(I)::value;
        v[z] = in[z];
    });
    fft<T, NP, -1>(v);
    const T s = (kx == N / 2 || ky == N / 2) ? T(0) : T(1.0 / ((double)NP * NP * NP));
    cx<T> u[N];
    sfor<N>([&](auto I) {
        constexpr int kz = decltype(I)::value;
        if constexpr (kz == N / 2) u[kz] = cx<T>{T(0), T(0)};
        else u[kz] = cx<T>{v[pad_pos<N, NP>(kz)].x * s, v[pad_pos<N, NP>(kz)].y * s};
    });
    fft<T, N, 1>(u);
    cx<T>* o = w2 + ((size_t)c * N * N + kx * N + ky) * N;
    sfor<N>([&](auto I) {
        constexpr int z = decltype(I)::value;
        o[z] = u[z];
    });
}

// x: inverse n-point transform over kx, real part -> q [x][y][z]
template <typename T, int N>
__global__ __launch_bounds__(128) void d_inv_x_re(const cx<T>* __restrict__ w2, T* __restrict__ q, int C) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= C * N * N) return;
    const int z = t % N, y = (t / N) % N, c = t / (N * N);
    const cx<T>* in = w2 + (size_t)c * N * N * N + y * N + z;
    cx<T> v[N];
    sfor<N>([&](auto I) {
        constexpr int k = decltype(I)::value;
        v[k] = in[k * N * N];
    });
    fft<T, N, 1>(v);
    T* o = q + (size_t)c * N * N * N + y * N + z;
    sfor<N>([&](auto I) {
        constexpr int x = decltype(I)::value;
        o[x * N * N] = v[x].x;
    });
}

inline size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

template <typename T, int N>
hipError_t run(const fks_plan* p, const fks_segment& s, void* ws, hipStream_t st) {
    constexpr int H = (N / 2 + 1) * N * N;
    constexpr size_t NN = (size_t)N * N * N;
    const int chunk = (int)std::min<int64_t>(s.ncell, chunk_cells(p, s.ncell));
    const int TB = terms_per_launch(p, s.ncell);
    char* base = (char*)ws;
    cx<T>* fh = (cx<T>*)base;
    cx<T>* work = (cx<T>*)(base + align256((size_t)chunk * H * sizeof(cx<T>)));
    const int64_t work_stride = (int64_t)(align256((size_t)chunk * NN * sizeof(cx<T>)) / sizeof(cx<T>));
    T* acc = (T*)(work + TB * work_stride);
    const cx<T>* tab = Tab<T>::get(p);
    const int bs = 128;
    for (int64_t c0 = 0; c0 < s.ncell; c0 += chunk) {
        const int C = (int)std::min<int64_t>(chunk, s.ncell - c0);
        const unsigned grid = (unsigned)((C * N * N + bs - 1) / bs);
        const double* f = s.f + c0 * (int64_t)NN;
        g_fwd_x<T, N><<<grid, bs, 0, st>>>(f, work, C);
        g_pass_y<T, N, -1><<<grid, bs, 0, st>>>(work, C);
        g_fwd_z<T, N><<<grid, bs, 0, st>>>(work, fh, C);
        constexpr int PP = zy_planes<N>();
        const unsigned gzy = (unsigned)(((int64_t)C * N + PP - 1) / PP);
        for (int j = 0; j < p->J; j += TB) {
            const int nt = std::min(TB, p->J - j);
            if constexpr (multi_term_ok<T, N>()) {
                g_inv_zy<T, N, true><<<gzy, PP * N, 0, st>>>(fh, tab + (size_t)j * H, work, C, nt, work_stride);
                g_inv_x<T, N, true><<<grid, bs, 0, st>>>(work, acc, C, j == 0 ? 1 : 0, nt, work_stride);
            } else {
                g_inv_zy<T, N, false><<<gzy, PP * N, 0, st>>>(fh, tab + (size_t)j * H, work, C, 1, work_stride);
                g_inv_x<T, N, false><<<grid, bs, 0, st>>>(work, acc, C, j == 0 ? 1 : 0, 1, work_stride);
            }
        }
        const double* fb = (s.f_base ? s.f_base : s.f) + c0 * (int64_t)NN;
        g_finish<T, N><<<C, 256, 0, st>>>(acc, fb, s.q_out ? s.q_out + c0 * (int64_t)NN : nullptr,
                                          s.f_out ? s.f_out + c0 * (int64_t)NN : nullptr, s.dt_over_tau, p->gc,
                                          p->d_guard, c0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// n-grid band index of a wavenumber index k' of the NP grid (FFT order), or -1 outside the band
// |k| < n/2 (the inverse of pad_pos)
template <int N, int NP>
__device__ __forceinline__ int band_of(int kp) {
    return kp < N / 2 ? kp : kp > NP - N / 2 ? kp - NP + N : -1;
}

// Band-limited data of the n grid, zero-padded to the NP grid in the layout of the NP = 48
// kernel: element (kz', kx', ky'), kz' < NP/2, of a slot of S complex at
// ((kz'/2) NP^2 + kx' NP + ky') 2 + kz' % 2; S = NP/2 NP^2 (tables) or (NP/2 + 1) NP^2
// (spectra, whose plane kz' = NP/2 stays zero).  Source: slots of H = (n/2+1) n^2 complex,
// element (kz, kx, ky) at (kz n + kx) n + ky.
template <int N, int NP>
__global__ __launch_bounds__(128) void d_embed48(const cx<float>* __restrict__ src, cx<float>* __restrict__ dst,
                                                 int64_t nslot, int S) {
    constexpr int H = (N / 2 + 1) * N * N, NN = NP * NP;
    const int64_t t = (int64_t)blockIdx.x * 128 + threadIdx.x;
    if (t >= nslot * S) return;
    const int64_t c = t / S;
    const int r = (int)(t - c * S);
    cx<float> v{0.0f, 0.0f};
    if (r < NP / 2 * NN) {
        const int m = r / (2 * NN), rem = r % (2 * NN), pos = rem / 2;
        const int kz = 2 * m + rem % 2, kx = band_of<N, NP>(pos / NP), ky = band_of<N, NP>(pos % NP);
        if (kz < N / 2 && kx >= 0 && ky >= 0) v = src[c * H + (kz * N + kx) * N + ky];
    }
    dst[t] = v;
}

struct DealiasLayout {
    size_t fh, w1, w2, acc, total;
};
template <typename T>
DealiasLayout dealias_layout(int n, int np, int chunk) {
    DealiasLayout L{};
    const size_t H = (size_t)(n / 2 + 1) * n * n;
    L.fh = 0;
    L.w1 = align256(chunk * H * sizeof(cx<T>));
    L.w2 = L.w1 + align256((size_t)chunk * n * n * np * sizeof(cx<T>));
    L.acc = L.w2 + align256((size_t)chunk * n * np * np * sizeof(cx<T>));
    L.total = L.acc + align256((size_t)chunk * np * np * np * sizeof(T));
    return L;
}

template <typename T, int N, int NP>
hipError_t run_dealias(const fks_plan* p, const fks_segment& s, void* ws, hipStream_t st) {
    static_assert(N * (size_t)N * N <= (size_t)N * NP * NP, "the n^3 stages reuse W2");
    constexpr int H = (N / 2 + 1) * N * N;
    constexpr size_t NN = (size_t)N * N * N;
    const int chunk = (int)std::min<int64_t>(s.ncell, chunk_cells(p, s.ncell));
    const DealiasLayout L = dealias_layout<T>(N, NP, chunk);
    char* base = (char*)ws;
    cx<T>* fh = (cx<T>*)(base + L.fh);
    cx<T>* w1 = (cx<T>*)(base + L.w1);
    cx<T>* w2 = (cx<T>*)(base + L.w2);
    T* acc = (T*)(base + L.acc);
    const cx<T>* tab = Tab<T>::get(p);
    const int bs = 128;
    auto grid = [&](int64_t threads) { return (unsigned)((threads + bs - 1) / bs); };
    for (int64_t c0 = 0; c0 < s.ncell; c0 += chunk) {
        const int C = (int)std::min<int64_t>(chunk, s.ncell - c0);
        // forward transform of f on the n grid (W2 as the n^3 work array)
        g_fwd_x<T, N><<<grid((int64_t)C * N * N), bs, 0, st>>>(s.f + c0 * (int64_t)NN, w2, C);
        g_pass_y<T, N, -1><<<grid((int64_t)C * N * N), bs, 0, st>>>(w2, C);
        g_fwd_z<T, N><<<grid((int64_t)C * N * N), bs, 0, st>>>(w2, fh, C);
        bool done = false;
        if constexpr (sizeof(T) == 4 && N == 32 && NP == 48) {
            if (p->d_tab48p) {
                // the NP = 48 kernel over the zero-padded spectrum (in W2) and tables: the same
                // products, transforms and Re z Im z on the 48-point grid, on chip
                constexpr int S = 25 * 48 * 48;
                d_embed48<N, NP><<<grid((int64_t)C * S), bs, 0, st>>>(fh, w2, C, S);
                const Piece48 pc{reinterpret_cast<const cx<float>*>(p->d_tab48p), 0, p->J};
                const hipError_t e = terms48(w2, &pc, 1, acc, C, reinterpret_cast<int*>(w1), p->grid48, st);
                if (e != hipSuccess) return e;
                done = true;
            }
        }
        for (int j = 0; j < p->J && !done; ++j) {
            d_term_zy<T, N, NP><<<(unsigned)(C * N), 64, 0, st>>>(fh, tab + (size_t)j * H, w2, C);
            d_pad_x<T, N, NP><<<grid((int64_t)C * NP * NP), bs, 0, st>>>(w2, acc, C, j == 0 ? 1 : 0);
        }
        // band coefficients of the products, back to the n grid
        d_trunc_x<T, N, NP><<<grid((int64_t)C * NP * NP), bs, 0, st>>>(acc, w2, C);
        d_trunc_y<T, N, NP><<<grid((int64_t)C * N * NP), bs, 0, st>>>(w2, w1, C);
        d_trunc_z_inv<T, N, NP><<<grid((int64_t)C * N * N), bs, 0, st>>>(w1, w2, C);
        g_pass_y<T, N, 1><<<grid((int64_t)C * N * N), bs, 0, st>>>(w2, C);
        d_inv_x_re<T, N><<<grid((int64_t)C * N * N), bs, 0, st>>>(w2, acc, C);
        const double* fb = (s.f_base ? s.f_base : s.f) + c0 * (int64_t)NN;
        g_finish<T, N><<<C, 256, 0, st>>>(acc, fb, s.q_out ? s.q_out + c0 * (int64_t)NN : nullptr,
                                          s.f_out ? s.f_out + c0 * (int64_t)NN : nullptr, s.dt_over_tau, p->gc,
                                          p->d_guard, c0);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename T>
hipError_t dispatch_dealias(const fks_plan* p, const fks_segment& s, void* ws, hipStream_t st) {
    switch (p->desc.n) {
        case 4: return run_dealias<T, 4, 6>(p, s, ws, st);
        case 8: return run_dealias<T, 8, 12>(p, s, ws, st);
        case 12: return run_dealias<T, 12, 18>(p, s, ws, st);
        case 16: return run_dealias<T, 16, 24>(p, s, ws, st);
        case 24: return run_dealias<T, 24, 36>(p, s, ws, st);
        case 32: return run_dealias<T, 32, 48>(p, s, ws, st);
        default: return hipErrorInvalidValue;
    }
}

template <typename T>
hipError_t dispatch(const fks_plan* p, const fks_segment& s, void* ws, hipStream_t st) {
    switch (p->desc.n) {
        case 4: return run<T, 4>(p, s, ws, st);
        case 6: return run<T, 6>(p, s, ws, st);
        case 8: return run<T, 8>(p, s, ws, st);
        case 12: return run<T, 12>(p, s, ws, st);
        case 16: return run<T, 16>(p, s, ws, st);
        case 24: return run<T, 24>(p, s, ws, st);
        case 32: return run<T, 32>(p, s, ws, st);
        case 48: return run<T, 48>(p, s, ws, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace

size_t generic_workspace_bytes(const fks_plan* p, int64_t ncell) {
    const int n = p->desc.n;
    if (p->desc.flags & FKS_FLAG_DEALIAS) {
        const int chunk = (int)std::min<int64_t>(std::max<int64_t>(ncell, 1), chunk_cells(p, ncell));
        return p->desc.precision == FKS_PREC_F64 ? dealias_layout<double>(n, 3 * n / 2, chunk).total
                                                 : dealias_layout<float>(n, 3 * n / 2, chunk).total;
    }
    const int chunk = (int)std::min<int64_t>(ncell, chunk_cells(p, ncell));
    const size_t TB = (size_t)terms_per_launch(p, ncell);
    size_t H = (size_t)(n / 2 + 1) * n * n, NN = (size_t)n * n * n;
    if (p->desc.precision == FKS_PREC_F64)
        return align256(chunk * H * sizeof(cx<double>)) + TB * align256(chunk * NN * sizeof(cx<double>)) +
               align256(chunk * NN * sizeof(double));
    return align256(chunk * H * sizeof(cx<float>)) + TB * align256(chunk * NN * sizeof(cx<float>)) +
           align256(chunk * NN * sizeof(float));
}

hipError_t embed_tables48(const fks_plan* p, hipStream_t st) {
    if (p->desc.n != 32 || !p->d_tab32 || !p->d_tab48p) return hipErrorInvalidValue;
    constexpr int S = 24 * 48 * 48;
    const int64_t total = (int64_t)p->J * S;
    d_embed48<32, 48><<<(unsigned)((total + 127) / 128), 128, 0, st>>>(
        reinterpret_cast<const cx<float>*>(p->d_tab32), reinterpret_cast<cx<float>*>(p->d_tab48p), p->J, S);
    return hipGetLastError();
}

hipError_t forward_f32_48(const double* f, cx<float>* work, cx<float>* fh, int C, hipStream_t st) {
    const int bs = 128;
    const unsigned grid = (unsigned)((C * 48 * 48 + bs - 1) / bs);
    g_fwd_x<float, 48><<<grid, bs, 0, st>>>(f, work, C);
    g_pass_y<float, 48, -1><<<grid, bs, 0, st>>>(work, C);
    g_fwd_z<float, 48, true><<<grid, bs, 0, st>>>(work, fh, C);
    return hipGetLastError();
}

size_t spectrum_workspace_bytes(int n, int64_t ncell) {
    const size_t chunk = (size_t)std::min<int64_t>(std::max<int64_t>(ncell, 1), kChunk);
    return chunk * (size_t)n * n * n * sizeof(cx<double>);
}

hipError_t spectrum(const double* x, double* xhat, int64_t ncell, int n, int zero_nyquist, void* ws, size_t ws_bytes,
                    hipStream_t st) {
    switch (n) {
        case 4: return run_spectrum<4>(x, xhat, ncell, zero_nyquist, ws, ws_bytes, st);
        case 6: return run_spectrum<6>(x, xhat, ncell, zero_nyquist, ws, ws_bytes, st);
        case 8: return run_spectrum<8>(x, xhat, ncell, zero_nyquist, ws, ws_bytes, st);
        case 12: return run_spectrum<12>(x, xhat, ncell, zero_nyquist, ws, ws_bytes, st);
        case 16: return run_spectrum<16>(x, xhat, ncell, zero_nyquist, ws, ws_bytes, st);
        case 24: return run_spectrum<24>(x, xhat, ncell, zero_nyquist, ws, ws_bytes, st);
        case 32: return run_spectrum<32>(x, xhat, ncell, zero_nyquist, ws, ws_bytes, st);
        case 48: return run_spectrum<48>(x, xhat, ncell, zero_nyquist, ws, ws_bytes, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t collide_generic(const fks_plan* p, const fks_segment& s, void* ws, size_t ws_bytes, hipStream_t st) {
    if (ws_bytes < generic_workspace_bytes(p, s.ncell)) return hipErrorInvalidValue;
    if (p->desc.flags & FKS_FLAG_DEALIAS) {
        if (p->desc.precision == FKS_PREC_F64) return dispatch_dealias<double>(p, s, ws, st);
        return dispatch_dealias<float>(p, s, ws, st);
    }
    if (p->desc.precision == FKS_PREC_F64) return dispatch<double>(p, s, ws, st);
    return dispatch<float>(p, s, ws, st);
}

}  // namespace fks
