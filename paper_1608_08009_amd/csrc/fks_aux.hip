// Moments (eq. i5 on the grid), the L2 projection onto prescribed moments
// (Section 3.2, eq. minim1), the FKS transport shift (Section 3.1 eq. f_bar,
// particle form of Section 4.1) and the halo messages of a z-slab decomposition
// of the grid (Section 4.2).  All FP64 and HBM-bound.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "fks_common.hpp"

namespace fks {
namespace {

constexpr int kBS = 256;
constexpr int kBcSlab = 2;   // z axis of a slab with ghost planes (not a public boundary condition)
typedef double d2v __attribute__((ext_vector_type(2)));

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

// source index along one axis of a destination index i shifted by sh: periodic wrap, or -1
// when a Dirichlet axis reaches outside (the inflow face), or the unwrapped index for the z
// axis of a slab (its ghost planes sit at -1 and nz)
__device__ __forceinline__ int source_index(int i, int sh, int dim, int bc, bool& outside) {
    int s = i - sh;
    if (bc == FKS_BC_PERIODIC) {
        if (s < 0) s += dim;   // one period covers every shift up to the axis length
        else if (s >= dim) s -= dim;
        if ((unsigned)s >= (unsigned)dim) {
            s %= dim;
            if (s < 0) s += dim;
        }
    } else if (bc != kBcSlab && (s < 0 || s >= dim)) {
        outside = true;
    }
    return s;
}

// q = k / n, r = k % n for 0 <= k < 2^24 and 1 <= n <= 64: the FP32 quotient is within one
// of the true one (k and n exact in FP32, one rounding), and one correction step fixes it
__device__ __forceinline__ void divmod_small(int k, int n, float inv_n, int& q, int& r) {
    q = (int)((float)k * inv_n);
    r = k - q * n;
    if (r < 0) {
        --q;
        r += n;
    } else if (r >= n) {
        ++q;
        r -= n;
    }
}

// out[iz][iy][ix][k] = in[iz - sz][iy - sy][ix - sx][k]   (periodic or Dirichlet inflow)
// One (x, y) column of cells per grid row (blockIdx.y, strided), walked along z, so the cell
// coordinates are uniform.  The z shift splits a velocity row (fixed kx, ky) of a source cell
// into up to three runs that land in three consecutive output cells of one column: walking
// the column keeps those reads on one CU, where the second and third runs hit the lines the
// first one brought into the cache.  A workgroup reads 4 KB per cell (U = 1), small enough
// that those lines are still there: cells in grid order fetched 2.3 to 3 times the
// algorithmic bytes, the column walk with 16 KB per cell (U = 4) 2.1 times, with 4 KB 1.35
// to 1.6 times.  Lanes run over a cell's velocities in groups of V consecutive kz (V = 2 for
// even n: 16-byte accesses where the two kz share their z shift, as they do everywhere
// except around v_z = 0).
template <int V, int U>
__global__ __launch_bounds__(kBS) void k_transport(const double* __restrict__ in, double* __restrict__ out,
                                                   int nx, int ny, int nz, int bcx, int bcy, int bcz, int n,
                                                   ShiftTable sh, const double* __restrict__ bc_f) {
    __shared__ int8_t sl[3][64];
    if (threadIdx.x < 3 * 64) sl[threadIdx.x / 64][threadIdx.x % 64] = sh.s[threadIdx.x / 64][threadIdx.x % 64];
    __syncthreads();
    const int nv = n * n * n;
    const int ngroup = nv / V;
    const int64_t ncol = (int64_t)nx * ny;
    const float inv_n = 1.0f / (float)n;
    for (int64_t col = blockIdx.y; col < ncol; col += gridDim.y)
    for (int iz = 0; iz < nz; ++iz) {
        const int ix = (int)(col % nx), iy = (int)(col / nx);
        const int64_t cell = iz * ncol + col;
        double v[U][V];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int g = (blockIdx.x * U + u) * kBS + threadIdx.x;
            if (g >= ngroup) break;
            const int k = g * V;
            int kxy, kz, kx, ky;
            divmod_small(k, n, inv_n, kxy, kz);
            divmod_small(kxy, n, inv_n, kx, ky);
            bool outx = false, outy = false;
            const int sx = source_index(ix, sl[0][kx], nx, bcx, outx);
            const int sy = source_index(iy, sl[1][ky], ny, bcy, outy);
#pragma unroll
            for (int e = 0; e < V; ++e) {
                bool outz = false;
                const int sz = source_index(iz, sl[2][kz + e], nz, bcz, outz);
                // the first out-of-range axis in x, y, z order decides the inflow face
                const int face = outx ? (sx < 0 ? 0 : 1) : outy ? (sy < 0 ? 2 : 3) : outz ? (sz < 0 ? 4 : 5) : -1;
                if (V == 2 && e == 0 && face < 0 && sl[2][kz] == sl[2][kz + 1]) {
                    // both kz from the same source cell: one 16-byte load
                    const double2 w = *reinterpret_cast<const double2*>(
                        in + (((int64_t)sz * ny + sy) * nx + sx) * nv + k);
                    v[u][0] = w.x;
                    v[u][V - 1] = w.y;
                    break;
                }
                v[u][e] = face >= 0 ? bc_f[(int64_t)face * nv + k + e]
                                    : in[(((int64_t)sz * ny + sy) * nx + sx) * nv + k + e];
            }
        }
        double* const o = out + cell * nv;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int g = (blockIdx.x * U + u) * kBS + threadIdx.x;
            if (g >= ngroup) break;
            if (V == 2) {
                __builtin_nontemporal_store(d2v{v[u][0], v[u][V - 1]}, reinterpret_cast<d2v*>(o + g * V));
            } else {
                __builtin_nontemporal_store(v[u][0], o + g);
            }
        }
    }
}

// Halo messages of a z slab: the n x n x h velocities of every cell of one plane whose
// kz lies in [k0, k0 + h), as buf[iy][ix][kx][ky][h].  pack copies them out of plane
// `plane` of f, unpack copies them into it; consecutive threads take consecutive buffer
// entries (coalesced writes for pack, coalesced reads for unpack; the f side is read or
// written in runs of h doubles).
template <bool PACK>
__global__ __launch_bounds__(kBS) void k_halo(double* __restrict__ f, double* __restrict__ buf, int64_t plane,
                                              int64_t ncell_plane, int n, int k0, int h) {
    const int64_t nv = (int64_t)n * n * n;
    const int64_t rows = ncell_plane * n * n;   // (cell, kx, ky) rows of the plane
    const int64_t total = rows * h;
    double* const base = f + plane * ncell_plane * nv;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = t / h;
        const int j = (int)(t - row * h);
        double* const g = base + row * n + k0 + j;   // row r = (cell, kx, ky): n^2 rows per cell
        if (PACK) buf[t] = *g;
        else *g = buf[t];
    }
}

}  // namespace

hipError_t halo_copy(double* f, double* buf, int64_t plane, int64_t ncell_plane, int n, int k0, int h, bool pack,
                     hipStream_t st) {
    const int64_t total = ncell_plane * n * n * h;
    if (total == 0) return hipSuccess;
    int64_t blocks = (total + kBS - 1) / kBS;
    if (blocks > 65536) blocks = 65536;
    if (pack) k_halo<true><<<(unsigned)blocks, kBS, 0, st>>>(f, buf, plane, ncell_plane, n, k0, h);
    else k_halo<false><<<(unsigned)blocks, kBS, 0, st>>>(f, buf, plane, ncell_plane, n, k0, h);
    return hipGetLastError();
}

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
                     const double* bc_f, hipStream_t st, bool slab) {
    // 16-byte accesses need even n and 16-byte aligned arrays (any double pointer is accepted)
    const bool aligned = ((uintptr_t)f_in | (uintptr_t)f_out | (uintptr_t)bc_f) % 16 == 0;
    const int V = (n % 2 == 0 && aligned) ? 2 : 1;
    constexpr int U = 1;
    const int ngroup = n * n * n / V;
    const int gx = (ngroup + kBS * U - 1) / (kBS * U);
    // one grid row per (x, y) column, up to about 32k workgroups in all
    const int64_t ncol = (int64_t)sp.nx * sp.ny;
    const unsigned gy = (unsigned)std::max<int64_t>(1, std::min<int64_t>({ncol, 65535, 32768 / gx}));
    const int bcz = slab ? kBcSlab : sp.bc[2];
    if (V == 2)
        k_transport<2, U><<<dim3((unsigned)gx, gy), kBS, 0, st>>>(f_in, f_out, sp.nx, sp.ny, sp.nz, sp.bc[0], sp.bc[1], bcz, n, sh,
                                                     bc_f);
    else
        k_transport<1, U><<<dim3((unsigned)gx, gy), kBS, 0, st>>>(f_in, f_out, sp.nx, sp.ny, sp.nz, sp.bc[0], sp.bc[1], bcz, n, sh,
                                                     bc_f);
    return hipGetLastError();
}

}  // namespace fks
