// Two velocity dimensions: the fast spectral operator for Maxwell molecules
// (Section 3.3, decoupled two-dimensional formula, eq. dfor0), one kernel per
// segment, FP64 or FP32 transforms with the FP64 conservation fix.
//
//   B_F(l, m) = w sum_p alpha_p(l) alpha'_p(m),  alpha_p(k) = phi(kappa k.e_p),
//   alpha'_p(k) = phi(kappa k.e_p^perp), phi(s) = 2R Sinc(Rs), t_p = pi p / A,
//   w = 2 C_0 pi / A.
//
// Per cell: fhat = n^-2 FFT(f) with the Nyquist lines zeroed; for each term
// (A gain terms, then the loss term) z = F^{-1}[(a + i b) fhat] and
// Q += Re z Im z, where (a, b) = (sqrt(w) alpha_p, sqrt(w) alpha'_p) for a gain
// term and (-L/s, s), s = sqrt(L(0)), for the loss term (Im z is then s f_N).
// Then the FP64 projection onto the kernel of (1, v_x, v_y, |v|^2)
// (eq. minim1) and the update f + dt/tau Q_c (eq. f_coll).
//
// Layout: n threads per cell, CPB cells per workgroup.  Thread i holds row
// x = i of the cell in the physical layout (registers over y) and column
// ky = i in the spectral layout (registers over kx); one LDS block of n rows
// (stride n+1) per cell turns one layout into the other, and also stages f and
// the outputs so that global loads and stores run along rows (coalesced).
#include <hip/hip_runtime.h>

#include <cmath>

#include "fks_fft.hpp"
#include "fks_internal.hpp"

namespace fks {

bool supported_n_2d(int n, int precision) {
    switch (n) {
        case 8: case 12: case 16: case 24: case 32: return true;
        case 48: case 64: return precision == FKS_PREC_F32_FIX64;
        default: return false;
    }
}

// Gram matrix of the scaled invariants over the n^2 grid, inverted in long double.
GridConst2 grid_const2(int n, double T) {
    GridConst2 g{};
    g.T = T;
    g.dv = 2.0 * T / n;
    long double G[4][4] = {};
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) {
            long double vx = (-T + i * g.dv) / T, vy = (-T + j * g.dv) / T;
            long double ph[4] = {1.0L, vx, vy, vx * vx + vy * vy};
            for (int a = 0; a < 4; ++a)
                for (int b = 0; b < 4; ++b) G[a][b] += ph[a] * ph[b];
        }
    long double M[4][8] = {};
    for (int a = 0; a < 4; ++a) {
        for (int b = 0; b < 4; ++b) M[a][b] = G[a][b];
        M[a][4 + a] = 1.0L;
    }
    for (int c = 0; c < 4; ++c) {
        int piv = c;
        for (int r = c + 1; r < 4; ++r)
            if (fabsl(M[r][c]) > fabsl(M[piv][c])) piv = r;
        for (int k = 0; k < 8; ++k) std::swap(M[c][k], M[piv][k]);
        long double d = M[c][c];
        for (int k = 0; k < 8; ++k) M[c][k] /= d;
        for (int r = 0; r < 4; ++r)
            if (r != c) {
                long double m = M[r][c];
                for (int k = 0; k < 8; ++k) M[r][k] -= m * M[c][k];
            }
    }
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b) g.ginv[a * 4 + b] = (double)M[a][4 + b];
    return g;
}

// Host FP64 tables of a dim = 2 plan, [J][n][n][2], k in FFT storage order.
void tables_2d(const fks_plan_desc& d, std::vector<double>& ab) {
    const int n = d.n, A = d.n_polar, J = A + 1;
    const double pi = 3.14159265358979323846;
    const double kappa = pi / d.T, R = d.R;
    const double w = 2.0 * d.c_gamma * pi / A, sw = std::sqrt(w);
    auto phi = [R](double s) {   // 2R Sinc(Rs)
        double x = R * s;
        return std::fabs(x) < 1e-8 ? 2.0 * R * (1.0 - x * x / 6.0) : 2.0 * R * std::sin(x) / x;
    };
    auto kw = [n](int i) { return i < n / 2 ? i : i - n; };
    ab.assign((size_t)J * n * n * 2, 0.0);
    std::vector<double> L((size_t)n * n, 0.0);
    for (int p = 1; p <= A; ++p) {
        const double t = pi * p / A, c = std::cos(t), s = std::sin(t);
        double* o = &ab[(size_t)(p - 1) * n * n * 2];
        for (int i = 0; i < n; ++i)
            for (int j = 0; j < n; ++j) {
                const double kx = kw(i), ky = kw(j);
                const double a = phi(kappa * (kx * c + ky * s));
                const double b = phi(kappa * (-kx * s + ky * c));
                o[((size_t)i * n + j) * 2] = sw * a;
                o[((size_t)i * n + j) * 2 + 1] = sw * b;
                L[(size_t)i * n + j] += w * a * b;
            }
    }
    const double sl = std::sqrt(L[0]);
    double* o = &ab[(size_t)A * n * n * 2];
    for (size_t k = 0; k < (size_t)n * n; ++k) {
        o[2 * k] = -L[k] / sl;
        o[2 * k + 1] = sl;
    }
}

namespace {

// Orders the LDS exchanges of one cell.  A cell's n threads are consecutive, so
// when n divides 64 they lie in one wave and a wave-level barrier suffices; for
// other n a cell can straddle two waves and the workgroup synchronises.
template <int N>
__device__ __forceinline__ void cell_sync() {
    if constexpr (64 % N == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    } else {
        __syncthreads();
    }
}

// LDS slot of a cell's block: 8 bytes, a complex value in FP32, a real value in FP64 (whose
// complex exchanges go through the block in two rounds, real parts then imaginary parts,
// which halves the block and doubles the cells a CU holds)
template <typename R>
struct Slot { using type = cx<float>; };
template <>
struct Slot<double> { using type = double; };

// cells per workgroup: n threads each, at most 256 threads and 128 KiB of LDS
template <typename R, int N>
constexpr int cells_per_block() {
    constexpr int by_threads = 256 / N;
    constexpr int by_lds = (128 * 1024) / (N * (N + 1) * (int)sizeof(typename Slot<R>::type));
    constexpr int c = by_threads < by_lds ? by_threads : by_lds;
    return c < 1 ? 1 : c;
}

struct Args2 {
    const double* f;
    double* q_out;
    double* f_out;
    const double* f_base;
    int64_t ncell;
    double dt;
    const void* tab;   // [J][N][N] pairs (a, b) in the transform type
    int J;
    const GridConst2* gc;
    unsigned long long* guard;   // numeric guard word, or null
};

template <typename R, int N>
__global__ __launch_bounds__((cells_per_block<R, N>() * N)) void k_collide2d(Args2 A) {
    constexpr int CPB = cells_per_block<R, N>();
    constexpr int RS = N + 1;
    constexpr int NN = N * N;
    using E = typename Slot<R>::type;
    static_assert(sizeof(E) == sizeof(double), "8-byte LDS slots");
    __shared__ E lds[CPB * N * RS];
    static_assert(N * 4 * sizeof(double) <= N * RS * sizeof(E), "reduction buffer inside a cell's block");
    const int t = threadIdx.x;
    const int c = t / N, i = t % N;
    const int64_t cell = (int64_t)blockIdx.x * CPB + c;
    const bool live = cell < A.ncell;
    E* const blk = lds + c * N * RS;
    // row layout -> column layout of one cell: src[k] of thread i lands in dst[i] of thread k
    auto transpose = [&](cx<R>(&src)[N], cx<R>(&dst)[N]) {
        if constexpr (sizeof(R) == 4) {
            sfor<N>([&](auto kI) { blk[decltype(kI)::value * RS + i] = src[decltype(kI)::value]; });
            cell_sync<N>();
            sfor<N>([&](auto kI) { dst[decltype(kI)::value] = blk[i * RS + decltype(kI)::value]; });
            cell_sync<N>();
        } else {
            sfor<N>([&](auto kI) { blk[decltype(kI)::value * RS + i] = src[decltype(kI)::value].x; });
            cell_sync<N>();
            sfor<N>([&](auto kI) { dst[decltype(kI)::value].x = blk[i * RS + decltype(kI)::value]; });
            cell_sync<N>();
            sfor<N>([&](auto kI) { blk[decltype(kI)::value * RS + i] = src[decltype(kI)::value].y; });
            cell_sync<N>();
            sfor<N>([&](auto kI) { dst[decltype(kI)::value].y = blk[i * RS + decltype(kI)::value]; });
            cell_sync<N>();
        }
    };
    const cx<R>* const tab = (const cx<R>*)A.tab;

    // ---- forward transform: row x = i over y, then columns over x ----
    // coalesced load: lane i reads element y = i of every row; the cell's block turns
    // the columns into rows.  The loads are unconditional (a past-the-end cell reads cell 0
    // and discards it): a load under the `live` condition is not speculated, and each then
    // waited for the memory before the next was issued.
    cx<R> z[N];
    {
        const double* fc = A.f + (live ? cell : 0) * (int64_t)NN + i;
        double fv[N];
        sfor<N>([&](auto xI) { fv[decltype(xI)::value] = fc[decltype(xI)::value * N]; });
        sfor<N>([&](auto xI) {
            constexpr int x = decltype(xI)::value;
            const R v = live ? (R)fv[x] : R(0);
            if constexpr (sizeof(R) == 4) blk[x * RS + i] = cx<float>{v, 0.0f};
            else blk[x * RS + i] = v;
        });
        cell_sync<N>();
        sfor<N>([&](auto yI) {
            constexpr int y = decltype(yI)::value;
            if constexpr (sizeof(R) == 4) z[y] = blk[i * RS + y];
            else z[y] = cx<R>{blk[i * RS + y], R(0)};
        });
        cell_sync<N>();
    }
    fft<R, N, -1>(z);
    cx<R> fh[N];   // column ky = i, registers over kx
    transpose(z, fh);
    fft<R, N, -1>(fh);
    {
        const R s = (i == N / 2) ? R(0) : R(1) / R(NN);
        sfor<N>([&](auto kI) {
            constexpr int k = decltype(kI)::value;
            const R sk = (k == N / 2) ? R(0) : s;
            fh[k] = cx<R>{fh[k].x * sk, fh[k].y * sk};
        });
    }

    // ---- terms: z = F^{-1}[(a + i b) fhat], Q += Re z Im z ----
    R q[N];
    sfor<N>([&](auto yI) { q[decltype(yI)::value] = R(0); });
    for (int j = 0; j < A.J; ++j) {
        const cx<R>* tj = tab + (size_t)j * NN + i;
        // (a, b) at (kx = k, ky = i), loaded in groups of kx, each group one scheduling
        // phase ahead of its products (left alone, the compiler waits on every load of
        // the FP64 kernel before issuing the next).  FP32 tables keep kx = 2m and 2m + 1
        // side by side (element (kx, ky) at ((kx/2) n + ky) 2 + kx % 2), so one 16-byte load
        // brings two kx: half the load instructions
        constexpr bool PAIRS = sizeof(R) == 4;
        constexpr int NG = PAIRS ? ((N / 2) % 4 == 0 ? 4 : (N / 2) % 3 == 0 ? 3 : 2) : (N % 4 == 0) ? 4 : 1;
        constexpr int GS = N / NG;
        static_assert(!PAIRS || GS % 2 == 0, "kx pairs per load group");
        cx<R> ab[N];
        sfor<NG + 1>([&](auto phI) {
            constexpr int ph = decltype(phI)::value;
            if constexpr (ph < NG && PAIRS)
                sfor<GS / 2>([&](auto mI) {
                    constexpr int m = ph * GS / 2 + decltype(mI)::value;
                    const float4 v = reinterpret_cast<const float4*>(tab + (size_t)j * NN)[m * N + i];
                    ab[2 * m] = cx<R>{v.x, v.y};
                    ab[2 * m + 1] = cx<R>{v.z, v.w};
                });
            if constexpr (ph < NG && !PAIRS)
                sfor<GS>([&](auto kI) {
                    constexpr int k = ph * GS + decltype(kI)::value;
                    ab[k] = tj[k * N];
                });
            if constexpr (ph > 0)
                sfor<GS>([&](auto kI) {
                    constexpr int k = (ph - 1) * GS + decltype(kI)::value;
                    z[k] = cx<R>{ab[k].x * fh[k].x - ab[k].y * fh[k].y, ab[k].x * fh[k].y + ab[k].y * fh[k].x};
                });
            __builtin_amdgcn_sched_barrier(0);
        });
        if constexpr (sizeof(R) == 4) {
            // over kx (column ky = i, registers over x), the transpose writes of each output
            // group leaving as the group is formed
            constexpr int R1 = first_radix<N>(), M1 = N / R1;
            fft_hook<R, N, 1>(z, [&](auto hI) {
                constexpr int h = decltype(hI)::value;
                if constexpr (h >= R1) {   // output group h - R1: x = h - R1 + M1 q
                    __builtin_amdgcn_sched_barrier(0);
                    sfor<R1>([&](auto qI) {
                        constexpr int x = h - R1 + M1 * decltype(qI)::value;
                        blk[x * RS + i] = z[x];
                    });
                    __builtin_amdgcn_sched_barrier(0);
                }
            });
            cell_sync<N>();
            sfor<N>([&](auto yI) { z[decltype(yI)::value] = blk[i * RS + decltype(yI)::value]; });
            cell_sync<N>();
        } else {
            fft<R, N, 1>(z);   // over kx: column ky = i, registers over x
            transpose(z, z);
        }
        fft<R, N, 1>(z);   // over ky: row x = i, registers over y
        sfor<N>([&](auto yI) {
            constexpr int y = decltype(yI)::value;
            q[y] = fma(z[y].x, z[y].y, q[y]);
        });
    }

    // ---- FP64 projection onto the kernel of (1, v_x, v_y, |v|^2) ----
    const GridConst2 g = *A.gc;
    const double h = g.dv / g.T;
    const double ux = -1.0 + i * h;
    double m[4] = {0.0, 0.0, 0.0, 0.0};
    sfor<N>([&](auto yI) {
        constexpr int y = decltype(yI)::value;
        const double uy = -1.0 + y * h, qq = (double)q[y];
        m[0] += qq;
        m[1] = fma(qq, ux, m[1]);
        m[2] = fma(qq, uy, m[2]);
        m[3] = fma(qq, fma(ux, ux, uy * uy), m[3]);
    });
    // the cell's own LDS block holds its partial sums: other cells (possibly in other
    // waves) may still be reading their blocks
    double* red = (double*)blk;
#pragma unroll
    for (int a = 0; a < 4; ++a) red[i * 4 + a] = m[a];
    cell_sync<N>();
    double s[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = 0; k < N; ++k)
#pragma unroll
        for (int a = 0; a < 4; ++a) s[a] += red[k * 4 + a];
    double lam[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        double v = 0.0;
#pragma unroll
        for (int b = 0; b < 4; ++b) v = fma(g.ginv[a * 4 + b], s[b], v);
        lam[a] = v;
    }
    if (live && A.guard && i == 0 && !isfinite(s[0] + s[1] + s[2] + s[3]))
        atomicMin(A.guard, (unsigned long long)cell);
    // Q_c of row x = i into the block (one double per slot), then coalesced stores: lane i
    // writes element y = i of every row
    constexpr int W = 1;   // one double per 8-byte slot
    double* const bd = (double*)blk;
    cell_sync<N>();   // every thread has read the partial sums
    const double lx = fma(lam[1], ux, lam[0]);
    sfor<N>([&](auto yI) {
        constexpr int y = decltype(yI)::value;
        const double uy = -1.0 + y * h;
        bd[(i * RS + y) * W] = (double)q[y] - (lx + lam[2] * uy + lam[3] * fma(ux, ux, uy * uy));
    });
    cell_sync<N>();
    if (!live) return;
    const int64_t base = cell * (int64_t)NN + i;
    if (A.f_out) {
        double fb[N];   // every load before the first store: f_out may alias f_base
        sfor<N>([&](auto xI) {
            constexpr int x = decltype(xI)::value;
            fb[x] = A.f_base[base + x * N];
        });
        sfor<N>([&](auto xI) {
            constexpr int x = decltype(xI)::value;
            const double qc = bd[(x * RS + i) * W];
            if (A.q_out) A.q_out[base + x * N] = qc;
            A.f_out[base + x * N] = fma(A.dt, qc, fb[x]);
        });
    } else {
        sfor<N>([&](auto xI) {
            constexpr int x = decltype(xI)::value;
            A.q_out[base + x * N] = bd[(x * RS + i) * W];
        });
    }
}

template <typename R, int N>
hipError_t launch2d(const Args2& a, hipStream_t st) {
    constexpr int CPB = cells_per_block<R, N>();
    const int64_t blocks = (a.ncell + CPB - 1) / CPB;
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    k_collide2d<R, N><<<(unsigned)blocks, CPB * N, 0, st>>>(a);
    return hipGetLastError();
}

template <typename R>
hipError_t dispatch2d(int n, const Args2& a, hipStream_t st) {
    switch (n) {
        case 8: return launch2d<R, 8>(a, st);
        case 12: return launch2d<R, 12>(a, st);
        case 16: return launch2d<R, 16>(a, st);
        case 24: return launch2d<R, 24>(a, st);
        case 32: return launch2d<R, 32>(a, st);
        default: break;
    }
    if constexpr (sizeof(R) == 4) {
        if (n == 48) return launch2d<R, 48>(a, st);
        if (n == 64) return launch2d<R, 64>(a, st);
    }
    return hipErrorInvalidValue;
}

}  // namespace

hipError_t collide_2d(const fks_plan* p, const fks_segment& s, hipStream_t st) {
    Args2 a{};
    a.f = s.f;
    a.q_out = s.q_out;
    a.f_out = s.f_out;
    a.f_base = s.f_base ? s.f_base : s.f;
    a.ncell = s.ncell;
    a.dt = s.dt_over_tau;
    a.J = p->J;
    a.gc = p->d_gc2;
    a.guard = p->d_guard;
    if (p->desc.precision == FKS_PREC_F64) {
        a.tab = p->d_tab64;
        return dispatch2d<double>(p->desc.n, a, st);
    }
    a.tab = p->d_tab32;
    return dispatch2d<float>(p->desc.n, a, st);
}

}  // namespace fks
