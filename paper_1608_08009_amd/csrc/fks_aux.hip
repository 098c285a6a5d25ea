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
typedef double d2v __attribute__((ext_vector_type(2)));

// Grid indices of i, i + kBS, i + 2 kBS, ... without a division per element: the first
// (x, y, z) by division, then steps of kBS = (dx, dy, dz) in mixed radix n with carries
// (dz, dy < n, so each carry is at most one).
struct Walk {
    int x, y, z, dx, dy, dz, n;
    __device__ Walk(int i, int n_) : n(n_) {
        z = i % n;
        y = (i / n) % n;
        x = i / (n * n);
        dz = kBS % n;
        dy = (kBS / n) % n;
        dx = kBS / (n * n);
    }
    __device__ __forceinline__ void step() {
        z += dz;
        int cy = 0;
        if (z >= n) {
            z -= n;
            cy = 1;
        }
        y += dy + cy;
        int cx = 0;
        if (y >= n) {
            y -= n;
            cx = 1;
        }
        x += dx + cx;
    }
};

// U[c] = dv^3 sum_j f_j (1, vx, vy, vz, |v|^2)
__global__ __launch_bounds__(kBS) void k_moments(const double* __restrict__ f, int n, GridConst gc,
                                                 double* __restrict__ U) {
    __shared__ double red[5 * (kBS / 64)];
    const int64_t c = blockIdx.x;
    const int nn = n * n * n;
    const double* fc = f + c * nn;
    double m[5] = {0, 0, 0, 0, 0};
    Walk w(threadIdx.x, n);
#pragma unroll 8   // eight loads in flight per thread: one at a time left the kernel latency-bound
    for (int i = threadIdx.x; i < nn; i += kBS, w.step()) {
        const double vx = fma((double)w.x, gc.dv, -gc.T), vy = fma((double)w.y, gc.dv, -gc.T),
                     vz = fma((double)w.z, gc.dv, -gc.T);
        const double v = fc[i];
        m[0] += v;
        m[1] = fma(v, vx, m[1]);
        m[2] = fma(v, vy, m[2]);
        m[3] = fma(v, vz, m[3]);
        m[4] = fma(v, fma(vx, vx, fma(vy, vy, vz * vz)), m[4]);
    }
    block_sum5<kBS>(m, red);
    if (threadIdx.x == 0) {
        const double dv3 = gc.dv * gc.dv * gc.dv;
        for (int a = 0; a < 5; ++a) U[c * 5 + a] = dv3 * m[a];
    }
}

// the scaled basis (1, v/T, |v|^2/T^2) at grid point (x, y, z); h = dv / T
__device__ __forceinline__ Basis scaled_basis(const Walk& w, double h) {
    const double ux = fma((double)w.x, h, -1.0), uy = fma((double)w.y, h, -1.0), uz = fma((double)w.z, h, -1.0);
    return Basis{{1.0, ux, uy, uz, fma(ux, ux, fma(uy, uy, uz * uz))}};
}

// f <- f + C^T (C C^T)^{-1} (U - C f), in the scaled basis
__global__ __launch_bounds__(kBS) void k_conserve(double* __restrict__ f, const double* __restrict__ U, int n,
                                                  GridConst gc) {
    __shared__ double red[5 * (kBS / 64)];
    __shared__ double lam_s[5];
    const int64_t c = blockIdx.x;
    const int nn = n * n * n;
    const double h = gc.dv / gc.T;
    double* fc = f + c * nn;
    double m[5] = {0, 0, 0, 0, 0};
    {
        Walk w(threadIdx.x, n);
#pragma unroll 8
        for (int i = threadIdx.x; i < nn; i += kBS, w.step()) {
            const Basis b = scaled_basis(w, h);
            const double v = fc[i];
#pragma unroll
            for (int a = 0; a < 5; ++a) m[a] = fma(v, b.p[a], m[a]);
        }
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
    Walk w(threadIdx.x, n);
#pragma unroll 8
    for (int i = threadIdx.x; i < nn; i += kBS, w.step()) fc[i] += correction(lam, scaled_basis(w, h));
}

// source index along one axis of a destination index i shifted by sh: periodic wrap, or
// `outside` when a Dirichlet axis reaches beyond the grid (the inflow face)
__device__ __forceinline__ int source_index(int i, int sh, int dim, int bc, bool& outside) {
    int s = i - sh;
    if (bc == FKS_BC_PERIODIC) {
        if (s < 0) s += dim;   // one period covers every shift up to the axis length
        else if (s >= dim) s -= dim;
        if ((unsigned)s >= (unsigned)dim) {
            s %= dim;
            if (s < 0) s += dim;
        }
    } else if (s < 0 || s >= dim) {
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

// Messages entering a z slab (layout [iy][ix][kx][ky][h], see k_halo): from below, the
// velocities with v_z > 0 (kz in [up0, up0 + hup)); from above, those with v_z < 0 (kz < hdn)
struct SlabIn {
    const double* below;
    const double* above;
    int up0, hup, hdn;
};

// out[iz][iy][ix][k] = in[iz - sz][iy - sy][ix - sx][k]   (periodic or Dirichlet inflow; in
// slab mode, source planes -1 and nz are the messages from the neighbours below and above)
// One (x, y) column of cells per grid row (blockIdx.y, strided), walked along z, so the cell
// coordinates are uniform.  The z shift splits a velocity row (fixed kx, ky) of a source cell
// into up to three runs that land in three consecutive output cells of one column: walking
// the column keeps those reads on one CU, where the second and third runs hit the lines the
// first one brought into the cache.  A workgroup reads 4 KB per cell, small enough that those
// lines are still there: on 32 x 32 x 32 cells of 24^3 velocities, cells in grid order fetched
// 2.3 to 3 times the algorithmic bytes, the column walk with 16 KB per cell 2.1 times, with
// 4 KB 1.07 to 1.21 times (1.24 to 1.28 on a 4-plane slab).  Lanes run over
// a cell's velocities in groups of V consecutive kz (V = 2 for even n: 16-byte accesses where
// the two kz share their source, as they do everywhere except around v_z = 0).
template <int V, bool SLAB>
__global__ __launch_bounds__(kBS) void k_transport(const double* __restrict__ in, double* __restrict__ out,
                                                   int nx, int ny, int nz, int bcx, int bcy, int bcz, int n,
                                                   ShiftTable sh, const double* __restrict__ bc_f, SlabIn msg) {
    __shared__ int8_t sl[3][64];
    if (threadIdx.x < 3 * 64) sl[threadIdx.x / 64][threadIdx.x % 64] = sh.s[threadIdx.x / 64][threadIdx.x % 64];
    __syncthreads();
    const int nv = n * n * n;
    const int ngroup = nv / V;
    const int64_t ncol = (int64_t)nx * ny;
    const float inv_n = 1.0f / (float)n;
    const int g = blockIdx.x * kBS + threadIdx.x;
    if (g >= ngroup) return;   // no barrier below
    const int k = g * V;
    int kxy, kz, kx, ky;
    divmod_small(k, n, inv_n, kxy, kz);
    divmod_small(kxy, n, inv_n, kx, ky);
    for (int64_t col = blockIdx.y; col < ncol; col += gridDim.y) {
        const int ix = (int)(col % nx), iy = (int)(col / nx);
        bool outx = false, outy = false;
        const int sx = source_index(ix, sl[0][kx], nx, bcx, outx);
        const int sy = source_index(iy, sl[1][ky], ny, bcy, outy);
        const int64_t src_col = (int64_t)sy * nx + sx;
        // one output cell: any source (cell, inflow face or neighbour's message), with branches
        auto one = [&](int iz) {
            double v[V];
#pragma unroll
            for (int e = 0; e < V; ++e) {
                bool outz = false;
                int sz;
                if (SLAB) sz = iz - sl[2][kz + e];   // -1 or nz: a neighbour's message
                else sz = source_index(iz, sl[2][kz + e], nz, bcz, outz);
                // the first out-of-range axis in x, y, z order decides the inflow face
                const int face = outx ? (sx < 0 ? 0 : 1) : outy ? (sy < 0 ? 2 : 3) : outz ? (sz < 0 ? 4 : 5) : -1;
                const bool inside = face < 0 && (!SLAB || (sz >= 0 && sz < nz));
                if (V == 2 && e == 0 && inside && sl[2][kz] == sl[2][kz + 1]) {
                    // both kz from the same source cell: one 16-byte load
                    const double2 w = *reinterpret_cast<const double2*>(in + (sz * ncol + src_col) * nv + k);
                    v[0] = w.x;
                    v[V - 1] = w.y;
                    break;
                }
                if (face >= 0) {
                    v[e] = bc_f[(int64_t)face * nv + k + e];
                } else if (inside) {
                    v[e] = in[(sz * ncol + src_col) * nv + k + e];
                } else {
                    const int64_t row = (src_col * n + kx) * n + ky;
                    v[e] = sz < 0 ? msg.below[row * msg.hup + (kz + e - msg.up0)] : msg.above[row * msg.hdn + kz + e];
                }
            }
            double* const o = out + (iz * ncol + col) * nv + k;
            if (V == 2) {
                __builtin_nontemporal_store(d2v{v[0], v[V - 1]}, reinterpret_cast<d2v*>(o));
            } else {
                __builtin_nontemporal_store(v[0], o);
            }
        };
        if constexpr (V == 1) {
            for (int iz = 0; iz < nz; ++iz) one(iz);
        } else {
            // Cells whose sources are cells of the grid or inflow faces (all of them, except a
            // slab's first and last plane, which read messages): the source of each kz is
            // selected without a branch and read with a 16-byte load of its aligned kz pair
            // (the two loads coincide when both kz share the source), so that the loads of
            // several cells are in flight together instead of one load, wait and store per cell.
            auto src = [&](int iz, int e) -> const double* {
                bool outz = false;
                const int sz = SLAB ? iz - sl[2][kz + e] : source_index(iz, sl[2][kz + e], nz, bcz, outz);
                const int face = outx ? (sx < 0 ? 0 : 1) : outy ? (sy < 0 ? 2 : 3) : outz ? (sz < 0 ? 4 : 5) : -1;
                return face >= 0 ? bc_f + (int64_t)face * nv + k : in + (sz * ncol + src_col) * nv + k;
            };
            int iz = 0;
            if (SLAB) one(iz++);
            const int iz_end = SLAB ? nz - 1 : nz;
            // cells [iz, iz_end) in groups of UU: the loads of a group, then its stores.  SAME:
            // both kz of every lane share their z shift, hence their source in every cell, and
            // one 16-byte load brings the pair
            auto run = [&](auto uI, auto sameI) {
                constexpr int UU = decltype(uI)::value;
                constexpr bool SAME = decltype(sameI)::value;
                for (; iz + UU <= iz_end; iz += UU) {
                    double2 a[UU], b[UU];
#pragma unroll
                    for (int u = 0; u < UU; ++u) {
                        a[u] = *reinterpret_cast<const double2*>(src(iz + u, 0));
                        if constexpr (!SAME) b[u] = *reinterpret_cast<const double2*>(src(iz + u, 1));
                    }
#pragma unroll
                    for (int u = 0; u < UU; ++u)
                        __builtin_nontemporal_store(d2v{a[u].x, SAME ? a[u].y : b[u].y},
                                                    reinterpret_cast<d2v*>(out + ((iz + u) * ncol + col) * nv + k));
                }
            };
            using I1 = std::integral_constant<int, 1>;
            using I2 = std::integral_constant<int, 2>;
            using I4 = std::integral_constant<int, 4>;
            if (__all(sl[2][kz] == sl[2][kz + 1])) {
                run(I4{}, std::true_type{});
                run(I2{}, std::true_type{});
                run(I1{}, std::true_type{});
            } else {
                run(I4{}, std::false_type{});
                run(I2{}, std::false_type{});
                run(I1{}, std::false_type{});
            }
            if (SLAB && nz > 1) one(nz - 1);
        }
    }
}

// Halo message of a z slab: the n x n x h velocities of every cell of one plane whose kz
// lies in [k0, k0 + h), as buf[iy][ix][kx][ky][h]; consecutive threads write consecutive
// buffer entries (the plane is read in runs of h doubles).
__global__ __launch_bounds__(kBS) void k_halo_pack(const double* __restrict__ f, double* __restrict__ buf,
                                                   int64_t plane, int64_t ncell_plane, int n, int k0, int h) {
    const int64_t nv = (int64_t)n * n * n;
    const int64_t rows = ncell_plane * n * n;   // (cell, kx, ky) rows of the plane
    const int64_t total = rows * h;
    const double* const base = f + plane * ncell_plane * nv;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total;
         t += (int64_t)gridDim.x * blockDim.x) {
        const int64_t row = t / h;
        const int j = (int)(t - row * h);
        buf[t] = base[row * n + k0 + j];   // row r = (cell, kx, ky): n^2 rows per cell
    }
}

}  // namespace

hipError_t halo_pack(const double* f, double* buf, int64_t plane, int64_t ncell_plane, int n, int k0, int h,
                     hipStream_t st) {
    const int64_t total = ncell_plane * n * n * h;
    if (total == 0) return hipSuccess;
    int64_t blocks = (total + kBS - 1) / kBS;
    if (blocks > 65536) blocks = 65536;
    k_halo_pack<<<(unsigned)blocks, kBS, 0, st>>>(f, buf, plane, ncell_plane, n, k0, h);
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
                     const double* bc_f, hipStream_t st, const double* from_below, const double* from_above) {
    // 16-byte accesses need even n and 16-byte aligned arrays (any double pointer is accepted)
    const bool aligned = ((uintptr_t)f_in | (uintptr_t)f_out | (uintptr_t)bc_f) % 16 == 0;
    const int V = (n % 2 == 0 && aligned) ? 2 : 1;
    const int ngroup = n * n * n / V;
    const int gx = (ngroup + kBS - 1) / kBS;
    // one grid row per (x, y) column, up to about 32k workgroups in all
    const int64_t ncol = (int64_t)sp.nx * sp.ny;
    const unsigned gy = (unsigned)std::max<int64_t>(1, std::min<int64_t>({ncol, 65535, 32768 / gx}));
    const bool slab = from_below != nullptr;
    const SlabIn msg{from_below, from_above, n / 2 + 1, n - 1 - n / 2, (n + 1) / 2};
    const dim3 grid((unsigned)gx, gy);
#define FKS_TRANSPORT(VV, SS)                                                                                 \
    k_transport<VV, SS><<<grid, kBS, 0, st>>>(f_in, f_out, sp.nx, sp.ny, sp.nz, sp.bc[0], sp.bc[1], sp.bc[2], n, \
                                              sh, bc_f, msg)
    if (V == 2 && slab) FKS_TRANSPORT(2, true);
    else if (V == 2) FKS_TRANSPORT(2, false);
    else if (slab) FKS_TRANSPORT(1, true);
    else FKS_TRANSPORT(1, false);
#undef FKS_TRANSPORT
    return hipGetLastError();
}

}  // namespace fks
