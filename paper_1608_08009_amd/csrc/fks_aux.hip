// Moments (eq. i5 on the grid), the L2 projection onto prescribed moments
// (Section 3.2, eq. minim1) and the FKS transport shift (Section 3.1 eq. f_bar,
// particle form of Section 4.1).  All FP64 and HBM-bound.
#include <hip/hip_runtime.h>

#include "fks_common.hpp"

namespace fks {
namespace {

constexpr int kBS = 256;

// U[c] = dv^3 sum_j f_j (1, vx, vy, vz, |v|^2)
__global__ __launch_bounds__(kBS) void k_moments(const double* __restrict__ f, int n, GridConst gc,
                                                 double* __restrict__ U) {
    __shared__ double red[5 * (kBS / 64)];
    const int64_t c = blockIdx.x;
    const int nn = n * n * n;
    const double* fc = f + c * nn;
    double m[5] = {0, 0, 0, 0, 0};
    for (int i = threadIdx.x; i < nn; i += kBS) {
        const int z = i % n, y = (i / n) % n, x = i / (n * n);
        const double vx = -gc.T + x * gc.dv, vy = -gc.T + y * gc.dv, vz = -gc.T + z * gc.dv;
        const double v = fc[i];
        m[0] += v;
        m[1] = fma(v, vx, m[1]);
        m[2] = fma(v, vy, m[2]);
        m[3] = fma(v, vz, m[3]);
        m[4] = fma(v, vx * vx + vy * vy + vz * vz, m[4]);
    }
    block_sum5<kBS>(m, red);
    if (threadIdx.x == 0) {
        const double dv3 = gc.dv * gc.dv * gc.dv;
        for (int a = 0; a < 5; ++a) U[c * 5 + a] = dv3 * m[a];
    }
}

// f <- f + C^T (C C^T)^{-1} (U - C f), in the scaled basis
__global__ __launch_bounds__(kBS) void k_conserve(double* __restrict__ f, const double* __restrict__ U, int n,
                                                  GridConst gc) {
    __shared__ double red[5 * (kBS / 64)];
    __shared__ double lam_s[5];
    const int64_t c = blockIdx.x;
    const int nn = n * n * n;
    double* fc = f + c * nn;
    double m[5] = {0, 0, 0, 0, 0};
    for (int i = threadIdx.x; i < nn; i += kBS) {
        const int z = i % n, y = (i / n) % n, x = i / (n * n);
        const Basis b = basis_at(gc, x, y, z);
        const double v = fc[i];
#pragma unroll
        for (int a = 0; a < 5; ++a) m[a] = fma(v, b.p[a], m[a]);
    }
    block_sum5<kBS>(m, red);
    if (threadIdx.x == 0) {
        const double idv3 = 1.0 / (gc.dv * gc.dv * gc.dv);
        const double tgt[5] = {U[c * 5] * idv3, U[c * 5 + 1] * idv3 / gc.T, U[c * 5 + 2] * idv3 / gc.T,
                               U[c * 5 + 3] * idv3 / gc.T, U[c * 5 + 4] * idv3 / (gc.T * gc.T)};
        double r[5], lam[5];
        for (int a = 0; a < 5; ++a) r[a] = tgt[a] - m[a];
        solve5(gc, r, lam);
        for (int a = 0; a < 5; ++a) lam_s[a] = lam[a];
    }
    __syncthreads();
    double lam[5];
#pragma unroll
    for (int a = 0; a < 5; ++a) lam[a] = lam_s[a];
    for (int i = threadIdx.x; i < nn; i += kBS) {
        const int z = i % n, y = (i / n) % n, x = i / (n * n);
        fc[i] += correction(lam, basis_at(gc, x, y, z));
    }
}

// out[iz][iy][ix][k] = in[iz - sz][iy - sy][ix - sx][k]   (periodic or Dirichlet inflow)
__global__ __launch_bounds__(kBS) void k_transport(const double* __restrict__ in, double* __restrict__ out,
                                                   int nx, int ny, int nz, int bcx, int bcy, int bcz, int n,
                                                   ShiftTable sh, const double* __restrict__ bc_f) {
    const int64_t nv = (int64_t)n * n * n;
    const int64_t total = (int64_t)nx * ny * nz * nv;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t cell = t / nv;
        const int k = (int)(t - cell * nv);
        const int kz = k % n, ky = (k / n) % n, kx = k / (n * n);
        const int ix = (int)(cell % nx), iy = (int)((cell / nx) % ny), iz = (int)(cell / ((int64_t)nx * ny));
        int sx = ix - sh.s[0][kx], sy = iy - sh.s[1][ky], sz = iz - sh.s[2][kz];
        int face = -1;
        if (bcx == FKS_BC_PERIODIC) {
            sx %= nx;
            if (sx < 0) sx += nx;
        } else if (sx < 0 || sx >= nx) {
            face = sx < 0 ? 0 : 1;
        }
        if (bcy == FKS_BC_PERIODIC) {
            sy %= ny;
            if (sy < 0) sy += ny;
        } else if (sy < 0 || sy >= ny) {
            if (face < 0) face = sy < 0 ? 2 : 3;
        }
        if (bcz == FKS_BC_PERIODIC) {
            sz %= nz;
            if (sz < 0) sz += nz;
        } else if (sz < 0 || sz >= nz) {
            if (face < 0) face = sz < 0 ? 4 : 5;
        }
        double v;
        if (face >= 0) {
            v = bc_f[(int64_t)face * nv + k];
        } else {
            v = in[(((int64_t)sz * ny + sy) * nx + sx) * nv + k];
        }
        out[t] = v;
    }
}

}  // namespace

hipError_t moments(const double* f, int64_t ncell, int n, double T, double* U, hipStream_t st) {
    GridConst gc = grid_const(n, T);
    k_moments<<<(unsigned)ncell, kBS, 0, st>>>(f, n, gc, U);
    return hipGetLastError();
}

hipError_t conserve(double* f, const double* U, int64_t ncell, int n, double T, hipStream_t st) {
    GridConst gc = grid_const(n, T);
    k_conserve<<<(unsigned)ncell, kBS, 0, st>>>(f, U, n, gc);
    return hipGetLastError();
}

hipError_t transport(const double* f_in, double* f_out, const fks_space_desc& sp, int n, const ShiftTable& sh,
                     const double* bc_f, hipStream_t st) {
    const int64_t total = (int64_t)sp.nx * sp.ny * sp.nz * n * n * n;
    int64_t blocks = (total + kBS - 1) / kBS;
    if (blocks > 65536) blocks = 65536;
    k_transport<<<(unsigned)blocks, kBS, 0, st>>>(f_in, f_out, sp.nx, sp.ny, sp.nz, sp.bc[0], sp.bc[1], sp.bc[2], n,
                                                 sh, bc_f);
    return hipGetLastError();
}

}  // namespace fks
