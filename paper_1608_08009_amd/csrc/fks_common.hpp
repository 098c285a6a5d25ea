// Device helpers shared by the collision kernels: grid coordinates, the
// FP64 projection onto the kernel of the collision invariants (Section 3.2,
// eq. minim1 applied to Q) and block reductions.
#pragma once

#include <hip/hip_runtime.h>

#include "fks_fft.hpp"
#include "fks_internal.hpp"

namespace fks {

// scaled invariants phi = (1, vx/T, vy/T, vz/T, |v|^2/T^2) at node (x, y, z)
struct Basis {
    double p[5];
};
__device__ __forceinline__ Basis basis_at(const GridConst& g, int x, int y, int z) {
    double vx = (-g.T + x * g.dv) / g.T, vy = (-g.T + y * g.dv) / g.T, vz = (-g.T + z * g.dv) / g.T;
    return Basis{{1.0, vx, vy, vz, vx * vx + vy * vy + vz * vz}};
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Sums m[0..4] over the block; result valid in every thread.  red: 5*NW doubles of LDS.
template <int NT>
__device__ __forceinline__ void block_sum5(double (&m)[5], double* red) {
    constexpr int NW = NT / 64;
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
#pragma unroll
    for (int a = 0; a < 5; ++a) m[a] = wave_sum(m[a]);
    if (l == 0) {
#pragma unroll
        for (int a = 0; a < 5; ++a) red[a * NW + w] = m[a];
    }
    __syncthreads();
#pragma unroll
    for (int a = 0; a < 5; ++a) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < NW; ++i) s += red[a * NW + i];
        m[a] = s;
    }
    __syncthreads();
}

// lambda = G^{-1} m
__device__ __forceinline__ void solve5(const GridConst& g, const double (&m)[5], double (&lam)[5]) {
#pragma unroll
    for (int a = 0; a < 5; ++a) {
        double s = 0.0;
#pragma unroll
        for (int b = 0; b < 5; ++b) s = fma(g.ginv[a * 5 + b], m[b], s);
        lam[a] = s;
    }
}

__device__ __forceinline__ double correction(const double (&lam)[5], const Basis& b) {
    return lam[0] * b.p[0] + lam[1] * b.p[1] + lam[2] * b.p[2] + lam[3] * b.p[3] + lam[4] * b.p[4];
}

}  // namespace fks
