// Fused FP32 collision kernel with FP64 conservation fix (one launch per batch).
//
// One workgroup owns one cell at a time (persistent loop over cells) and keeps
// the whole n^3 complex working set of a transform on chip: every thread holds
// P pencils of n complex values in registers, and the two transposes of each
// 3D transform go through LDS.  Per cell:
//   1. f (FP64, HBM) -> FP32, forward 3D FFT, scale n^-3, zero the Nyquist
//      planes, store the half spectrum kz in [0, n/2] in a per-workgroup slot
//      (L2-resident workspace)                                      (eq. FC)
//   2. for each term j (M*K gain terms, then the loss term (-L, 1)):
//      Z = (a_j + i b_j) fhat (mirror + conjugate for kz > n/2), inverse 3D
//      FFT, Q += Re(z) Im(z) in registers                          (eq. ode, fast form)
//   3. FP64: moments of Q, lambda = G^{-1} C Q, Q_c = Q - C^T lambda,
//      q_out = Q_c and/or f_out = f + dt/tau Q_c                   (eqs. minim1, f_coll)
//
// Thread layouts (t = hi * n + lo, hi in [0, n/P), HP = n/P; pencil p in [0, P)):
//   C: pencil (y = hi + HP p, z = lo), registers over x      (physical side)
//   B: pencil (kx = hi + HP p, z = lo), registers over y
//   A: pencil (kx = hi + HP p, ky = lo), registers over kz   (spectral side)
// LDS holds HP blocks of n rows with row stride n+1 (padding against bank
// conflicts; every LDS access is a per-thread base plus an immediate offset).
// A <-> B only swaps (lane, register) inside the n threads sharing hi: it goes
// through that group's own block and needs no workgroup barrier.  B <-> C
// crosses waves: P rounds of n^3/P^2 values with workgroup barriers; in round
// r each group reads back only its own block, so the next group-local
// exchange can reuse that block without a barrier.
#include <hip/hip_runtime.h>

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
struct Cfg<32> { static constexpr int P = 2; };

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
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

template <int N>
__global__ __launch_bounds__(N * N / Cfg<N>::P) void k_fused(const double* f, double* __restrict__ q_out,
                                                            double* f_out, int64_t ncell, double dt,
                                                            const cx<float>* __restrict__ tab, int J,
                                                            cx<float>* __restrict__ fh_ws,
                                                            const GridConst* __restrict__ gcp) {
    constexpr int P = Cfg<N>::P;
    constexpr int NT = N * N / P;
    constexpr int HP = N / P;
    constexpr int NN = N * N;
    constexpr int RS = N + 1;        // LDS row stride (complex)
    constexpr int BS = N * RS;       // LDS block stride
    constexpr int H = (N / 2 + 1) * N * N;
    __shared__ cx<float> lds[HP * BS];
    __shared__ double red[5 * (NT / 64 > 0 ? NT / 64 : 1)];

    const int t = threadIdx.x;
    const int hi = t / N, lo = t % N;
    cx<float>* const blk = lds + hi * BS;   // this group's block
    cx<float>* const fh = fh_ws + (size_t)blockIdx.x * H;

    for (int64_t cell = blockIdx.x; cell < ncell; cell += gridDim.x) {
        const double* fc = f + cell * (int64_t)(NN * N);

        // ---------------- forward transform ----------------
        cx<float> c[P][N];
        sfor<P>([&](auto pI) {
            constexpr int p = decltype(pI)::value;
            const double* src = fc + opaque((hi + HP * p) * N + lo);
            sfor<N>([&](auto xI) {
                constexpr int x = decltype(xI)::value;
                c[p][x] = cx<float>{(float)src[x * NN], 0.0f};
            });
            fft<float, N, -1>(c[p]);
        });
        cx<float> b[P][N];
        sfor<P>([&](auto rI) {   // C -> B, round r delivers B-pencil r (kx in [HP r, HP r + HP))
            constexpr int r = decltype(rI)::value;
            __syncthreads();
            sfor<P>([&](auto pI) {
                constexpr int p = decltype(pI)::value;
                cx<float>* dst = lds + (hi + HP * p) * RS + lo;   // row y, column z
                sfor<HP>([&](auto xI) {
                    constexpr int xx = decltype(xI)::value;
                    dst[xx * BS] = c[p][HP * r + xx];
                });
            });
            __syncthreads();
            sfor<N>([&](auto yI) {
                constexpr int y = decltype(yI)::value;
                b[r][y] = blk[y * RS + lo];
            });
        });
        cx<float> a[P][N];
        sfor<P>([&](auto pI) {
            constexpr int p = decltype(pI)::value;
            fft<float, N, -1>(b[p]);
            // B -> A inside the group: element (row ky, column z)
            sfor<N>([&](auto kI) {
                constexpr int ky = decltype(kI)::value;
                blk[ky * RS + lo] = b[p][ky];
            });
            wave_sync();
            sfor<N>([&](auto zI) {
                constexpr int z = decltype(zI)::value;
                a[p][z] = blk[lo * RS + z];
            });
            wave_sync();
            fft<float, N, -1>(a[p]);
            const int kx = hi + HP * p;
            const float s = ((kx == N / 2) || (lo == N / 2)) ? 0.0f : 1.0f / (float)(N * N * N);
            cx<float>* o = fh + opaque(kx * N + lo);
            sfor<N / 2>([&](auto kI) {
                constexpr int kz = decltype(kI)::value;
                o[kz * NN] = cx<float>{a[p][kz].x * s, a[p][kz].y * s};
            });
            o[(N / 2) * NN] = cx<float>{0.0f, 0.0f};
        });
        __threadfence_block();
        __syncthreads();

        // ---------------- terms ----------------
        float q[P][N];
        sfor<P>([&](auto pI) {
            constexpr int p = decltype(pI)::value;
            sfor<N>([&](auto xI) { q[p][decltype(xI)::value] = 0.0f; });
        });
        for (int j = 0; j < J; ++j) {
            const cx<float>* tj = tab + (size_t)j * H;
            cx<float> za[P][N];
            sfor<P>([&](auto pI) {
                constexpr int p = decltype(pI)::value;
                const int kx = hi + HP * p;
                const int o1 = opaque(kx * N + lo);
                const int o2 = opaque(((N - kx) & (N - 1)) * N + ((N - lo) & (N - 1)));
                sfor<N>([&](auto kI) {
                    constexpr int kz = decltype(kI)::value;
                    if constexpr (kz <= N / 2) {
                        const int h = o1 + kz * NN;
                        za[p][kz] = cmulf(tj[h], fh[h]);
                    } else {
                        const int h = o2 + (N - kz) * NN;
                        cx<float> g = fh[h];
                        g.y = -g.y;
                        za[p][kz] = cmulf(tj[h], g);
                    }
                });
                fft<float, N, 1>(za[p]);
            });
            cx<float> zb[P][N];
            sfor<P>([&](auto pI) {   // A -> B inside the group
                constexpr int p = decltype(pI)::value;
                sfor<N>([&](auto zI) {
                    constexpr int z = decltype(zI)::value;
                    blk[lo * RS + z] = za[p][z];
                });
                wave_sync();
                sfor<N>([&](auto kI) {
                    constexpr int ky = decltype(kI)::value;
                    zb[p][ky] = blk[ky * RS + lo];
                });
                wave_sync();
                fft<float, N, 1>(zb[p]);
            });
            cx<float> zc[P][N];
            sfor<P>([&](auto rI) {   // B -> C, round r delivers C-pencil r (y in [HP r, HP r + HP))
                constexpr int r = decltype(rI)::value;
                __syncthreads();
                sfor<P>([&](auto pI) {
                    constexpr int p = decltype(pI)::value;
                    cx<float>* dst = lds + (hi + HP * p) * RS + lo;   // row kx, column z
                    sfor<HP>([&](auto yI) {
                        constexpr int yy = decltype(yI)::value;
                        dst[yy * BS] = zb[p][HP * r + yy];
                    });
                });
                __syncthreads();
                sfor<N>([&](auto kI) {
                    constexpr int kx = decltype(kI)::value;
                    zc[r][kx] = blk[kx * RS + lo];
                });
            });
            sfor<P>([&](auto pI) {
                constexpr int p = decltype(pI)::value;
                fft<float, N, 1>(zc[p]);
                sfor<N>([&](auto xI) {
                    constexpr int x = decltype(xI)::value;
                    q[p][x] = fmaf(zc[p][x].x, zc[p][x].y, q[p][x]);
                });
            });
        }

        // ---------------- FP64 projection and update ----------------
        // scaled invariants (1, vx/T, vy/T, vz/T, |v|^2/T^2); the grid step is
        // made opaque so the per-node coordinates are not hoisted out of the
        // cell loop into long-lived registers
        const double h = opaque(gcp->dv / gcp->T);
        const double uz = -1.0 + lo * h;
        double m[5] = {0, 0, 0, 0, 0};
        sfor<P>([&](auto pI) {
            constexpr int p = decltype(pI)::value;
            const double uy = -1.0 + (hi + HP * p) * h;
            const double r2 = uy * uy + uz * uz;
            sfor<N>([&](auto xI) {
                constexpr int x = decltype(xI)::value;
                const double ux = -1.0 + x * h;
                const double qv = (double)q[p][x];
                m[0] += qv;
                m[1] = fma(qv, ux, m[1]);
                m[2] = fma(qv, uy, m[2]);
                m[3] = fma(qv, uz, m[3]);
                m[4] = fma(qv, fma(ux, ux, r2), m[4]);
            });
        });
        block_sum5<NT>(m, red);
        double lam[5];
        solve5(*gcp, m, lam);
        const int64_t base = cell * (int64_t)(NN * N);
        sfor<P>([&](auto pI) {
            constexpr int p = decltype(pI)::value;
            const double uy = -1.0 + (hi + HP * p) * h;
            const double r2 = uy * uy + uz * uz;
            const double l0 = lam[0] + lam[2] * uy + lam[3] * uz + lam[4] * r2;
            const int64_t off = base + opaque((hi + HP * p) * N + lo);
            double qc[N];
            sfor<N>([&](auto xI) {
                constexpr int x = decltype(xI)::value;
                const double ux = -1.0 + x * h;
                qc[x] = (double)q[p][x] - fma(lam[4], ux * ux, fma(lam[1], ux, l0));
            });
            if (q_out) {
                sfor<N>([&](auto xI) {
                    constexpr int x = decltype(xI)::value;
                    q_out[off + x * NN] = qc[x];
                });
            }
            if (f_out) {
                sfor<N>([&](auto xI) {
                    constexpr int x = decltype(xI)::value;
                    f_out[off + x * NN] = fma(dt, qc[x], f[off + x * NN]);
                });
            }
        });
    }
}

template <int N>
int grid_for(int device) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess || cus <= 0)
        cus = 256;
    int per = 0;
    constexpr int NT = N * N / Cfg<N>::P;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_fused<N>, NT, 0) != hipSuccess || per <= 0) per = 1;
    return cus * per;
}

template <int N>
hipError_t launch(const fks_plan* p, const fks_segment& s, void* ws, hipStream_t st) {
    constexpr int NT = N * N / Cfg<N>::P;
    const int64_t grid = std::min<int64_t>(s.ncell, p->fused_grid);
    k_fused<N><<<(unsigned)grid, NT, 0, st>>>(s.f, s.q_out, s.f_out, s.ncell, s.dt_over_tau,
                                             reinterpret_cast<const cx<float>*>(p->d_tab32), p->J,
                                             reinterpret_cast<cx<float>*>(ws), p->d_gc);
    return hipGetLastError();
}

}  // namespace

bool fused_available(int n) { return n == 8 || n == 16 || n == 32; }

int fused_grid_size(int n, int device) {
    switch (n) {
        case 8: return grid_for<8>(device);
        case 16: return grid_for<16>(device);
        case 32: return grid_for<32>(device);
        default: return 0;
    }
}

size_t fused_workspace_bytes(const fks_plan* p, int64_t ncell) {
    const int n = p->desc.n;
    const int64_t grid = std::min<int64_t>(ncell, p->fused_grid);
    return (size_t)grid * (size_t)(n / 2 + 1) * n * n * sizeof(cx<float>);
}

hipError_t collide_fused(const fks_plan* p, const fks_segment& s, void* ws, size_t ws_bytes, hipStream_t st) {
    if (ws_bytes < fused_workspace_bytes(p, s.ncell)) return hipErrorInvalidValue;
    switch (p->desc.n) {
        case 8: return launch<8>(p, s, ws, st);
        case 16: return launch<16>(p, s, ws, st);
        case 32: return launch<32>(p, s, ws, st);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace fks
