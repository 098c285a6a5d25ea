// BGK relaxation operator with the conservative discrete Maxwellian
// (Section 2 eq. ibgk; Section 3.2 eq. minimMax), FP64, one workgroup per cell.
//
//   U = C f; (rho, u, theta) from U with d rho theta = sum |v|^2 f dv^d - rho |u|^2;
//   M~ = rho (2 pi theta)^{-d/2} exp(-|v - u|^2 / (2 theta)) at the nodes;
//   E = M~ + C^T (C C^T)^{-1} (U - C M~)   (so C E = U);
//   Q = nu' (E - f), nu' = nu or nu * rho;
//   f_out = f + (dt/tau) Q (eq. f_coll) or E + exp(-nu' dt/tau) (f - E).
//
// The projection is taken in the scaled basis (1, v/T, |v|^2/T^2), where it
// reads E = M~ + phi^T G^{-1} (phi f - phi M~) with G the Gram matrix of the
// scaled basis over the grid.  The Maxwellian factorises over the axes: the
// 1D factors live in LDS, and the moments of M~ over the grid are products of
// 1D sums S_a,p = sum_j g_a[j] u_j^p (p = 0, 1, 2), so no pass over the grid
// is needed for them.  Cells of up to 32 rows of two nodes per thread (512
// threads, even n: n^3 <= 32768, n^2 <= 16384) keep f in registers (k_bgk_reg:
// one HBM read and one write per node); larger cells read f twice (k_bgk), the
// second time mostly from the caches.
#include <hip/hip_runtime.h>

#include <cmath>

#include "fks_internal.hpp"

namespace fks {
namespace {

#ifndef FKS_BGK_THREADS
#define FKS_BGK_THREADS 512
#endif
constexpr int kBgkThreads = FKS_BGK_THREADS;   // threads per workgroup (one cell)
#ifndef FKS_BGK_MAXROWS
#define FKS_BGK_MAXROWS 32
#endif
constexpr int kBgkMaxRows = FKS_BGK_MAXROWS;   // rows per thread kept in registers
#ifndef FKS_BGK_UNROLL
#define FKS_BGK_UNROLL 4
#endif

struct BgkArgs {
    const double* f;
    double* q_out;
    double* f_out;
    int64_t ncell;
    int n;
    double T;
    double dv;
    double nu;
    int nu_rho;
    int exact;
    double dt;
    double ginv[25];   // inverse Gram matrix of the scaled basis (dim + 2 rows used)
};

// hides a value from common-subexpression elimination across the reduction, so
// that node coordinates are recomputed instead of held in registers
__device__ __forceinline__ int bgk_opaque(int v) {
    asm volatile("" : "+v"(v));
    return v;
}

__device__ __forceinline__ double bgk_wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// sums m[0..K-1] over the workgroup (all threads get the result); red: K * 16 doubles
template <int K>
__device__ __forceinline__ void bgk_block_sum(double (&m)[K], double* red) {
    const int w = threadIdx.x >> 6, l = threadIdx.x & 63, nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int a = 0; a < K; ++a) m[a] = bgk_wave_sum(m[a]);
    if (l == 0)
#pragma unroll
        for (int a = 0; a < K; ++a) red[a * 16 + w] = m[a];
    __syncthreads();
#pragma unroll
    for (int a = 0; a < K; ++a) {
        double s = 0.0;
        for (int i = 0; i < nw; ++i) s += red[a * 16 + i];
        m[a] = s;
    }
    __syncthreads();
}

// Primitive variables from the scaled moments m, the 1D factors g1 and the
// moments mm of the pointwise Maxwellian (from the 1D sums), the multipliers
// lam = G^{-1} (m - mm).  Called by every thread of the workgroup; ok = false
// (and lam = 0) for a cell without a Maxwellian.
template <int D>
struct MaxwellFit {
    double pref;       // rho (2 pi theta)^{-d/2}
    double nup;        // nu'
    double lam[D + 2];
    bool ok;
};

template <int D>
__device__ __forceinline__ MaxwellFit<D> fit_maxwellian(const BgkArgs& A, const double (&m)[D + 2],
                                                        double (*g1)[512], double* S) {
    constexpr int K = D + 2;
    const int n = A.n, t = threadIdx.x, nt = blockDim.x;
    MaxwellFit<D> r{};
    double vol = 1.0;
#pragma unroll
    for (int a = 0; a < D; ++a) vol *= A.dv;
    const double rho = vol * m[0];
    double u[D], u2 = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
        u[a] = A.T * m[1 + a] / m[0];
        u2 += u[a] * u[a];
    }
    const double theta = (A.T * A.T * m[K - 1] / m[0] - u2) / D;
    r.ok = rho > 0.0 && theta > 0.0 && isfinite(theta) && isfinite(rho);
    r.nup = A.nu_rho ? A.nu * rho : A.nu;
    if (r.ok) {
        for (int i = t; i < D * n; i += nt) {
            const int a = i / n, j = i % n;
            const double d = -A.T + j * A.dv - u[a];
            g1[a][j] = exp(-d * d / (2.0 * theta));
        }
        const double tp = 2.0 * 3.14159265358979323846 * theta;
        r.pref = rho / (D == 3 ? tp * sqrt(tp) : tp);
    }
    __syncthreads();
    // 1D sums S[a][p] = sum_j g_a[j] u_j^p, one wave per axis
    const int w = t >> 6, l = t & 63;
    if (r.ok && w < D) {
        const double h = A.dv / A.T;
        double s0 = 0.0, s1 = 0.0, s2 = 0.0;
        for (int j = l; j < n; j += 64) {
            const double g = g1[w][j], uj = -1.0 + j * h;
            s0 += g;
            s1 = fma(g, uj, s1);
            s2 = fma(g * uj, uj, s2);
        }
        s0 = bgk_wave_sum(s0);
        s1 = bgk_wave_sum(s1);
        s2 = bgk_wave_sum(s2);
        if (l == 0) {
            S[w * 3 + 0] = s0;
            S[w * 3 + 1] = s1;
            S[w * 3 + 2] = s2;
        }
    }
    __syncthreads();
    double mm[K];
#pragma unroll
    for (int a = 0; a < K; ++a) mm[a] = 0.0;
    if (r.ok) {
        // mm_0 = c prod_a S_a0; mm_{1+a} = c S_a1 prod_{b != a} S_b0;
        // mm_{K-1} = c sum_a S_a2 prod_{b != a} S_b0
        double p0 = r.pref;
#pragma unroll
        for (int a = 0; a < D; ++a) p0 *= S[a * 3];
        mm[0] = p0;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            double o = r.pref;
#pragma unroll
            for (int b = 0; b < D; ++b)
                if (b != a) o *= S[b * 3];
            mm[1 + a] = o * S[a * 3 + 1];
            mm[K - 1] = fma(o, S[a * 3 + 2], mm[K - 1]);
        }
    }
#pragma unroll
    for (int a = 0; a < K; ++a) {
        double s = 0.0;
#pragma unroll
        for (int b = 0; b < K; ++b) s = fma(A.ginv[a * K + b], m[b] - mm[b], s);
        r.lam[a] = r.ok ? s : 0.0;
    }
    return r;
}

// Node layout of one cell: the n nodes of a row (last index z) form n/W groups
// of W consecutive nodes (W = 2 for even n: 16-byte accesses); thread t owns
// the group starting at z = W (t mod n/W) and the rows r = t / (n/W) + k rstep,
// rstep = nt / (n/W); row r is (x, y) = (r / n, r mod n) in three dimensions and
// x = r in two.  The walk over a thread's rows advances (x, y) by
// (rstep / n, rstep mod n) with one carry, so no division is needed per row.
template <int D, int W>
struct Rows {
    int n, z, r0, rstep, rows, x0, y0, dx, dy;
    __device__ explicit Rows(int n_) : n(n_) {
        const int cg = n / W;
        z = (threadIdx.x % cg) * W;
        r0 = threadIdx.x / cg;
        rstep = blockDim.x / cg;
        rows = D == 3 ? n * n : n;
        if (D == 3) {
            x0 = r0 / n;
            y0 = r0 % n;
            dx = rstep / n;
            dy = rstep % n;
        } else {
            x0 = r0;
            y0 = 0;
            dx = rstep;
            dy = 0;
        }
    }
    __device__ __forceinline__ void next(int& x, int& y) const {
        x += dx;
        y += dy;
        if (D == 3 && y >= n) {
            y -= n;
            x += 1;
        }
    }
};

typedef double d2v __attribute__((ext_vector_type(2)));

template <int W, bool NT>
__device__ __forceinline__ void load_w(const double* p, double (&o)[W]) {
    if constexpr (W == 2) {
        const d2v v = NT ? __builtin_nontemporal_load((const d2v*)p) : *(const d2v*)p;
        o[0] = v[0];
        o[1] = v[1];
    } else {
        o[0] = NT ? __builtin_nontemporal_load(p) : *p;
    }
}
template <int W>
__device__ __forceinline__ void store_w(double* p, const double (&v)[W]) {
    if constexpr (W == 2) __builtin_nontemporal_store(d2v{v[0], v[1]}, (d2v*)p);
    else __builtin_nontemporal_store(v[0], p);
}

// scaled moments (1, u_x, [u_y,] u_z, |u|^2) of one node value
template <int D>
__device__ __forceinline__ void add_moments(double (&m)[D + 2], double f, double ux, double uy, double uz) {
    m[0] += f;
    m[1] = fma(f, ux, m[1]);
    if (D == 3) {
        m[2] = fma(f, uy, m[2]);
        m[3] = fma(f, uz, m[3]);
        m[4] = fma(f, fma(ux, ux, fma(uy, uy, uz * uz)), m[4]);
    } else {
        m[2] = fma(f, uz, m[2]);
        m[3] = fma(f, fma(ux, ux, uz * uz), m[3]);
    }
}

// E at node (x, y, z) for a fitted cell
template <int D>
__device__ __forceinline__ double equilibrium(const MaxwellFit<D>& F, double (*g1)[512], double gz, int x, int y,
                                              double ux, double uy, double uz) {
    double mv = F.pref * g1[0][x] * gz;
    if (D == 3) {
        mv *= g1[1][y];
        return mv + (F.lam[0] + F.lam[1] * ux + F.lam[2] * uy + F.lam[3] * uz +
                     F.lam[4] * fma(ux, ux, fma(uy, uy, uz * uz)));
    }
    return mv + (F.lam[0] + F.lam[1] * ux + F.lam[2] * uz + F.lam[3] * fma(ux, ux, uz * uz));
}

// outputs of one group of W nodes
template <int D, int W>
__device__ __forceinline__ void emit(const BgkArgs& A, const MaxwellFit<D>& F, double (*g1)[512], int64_t idx,
                                     const double (&f)[W], int x, int y, int z, double h, double decay) {
    double q[W], o[W];
#pragma unroll
    for (int c = 0; c < W; ++c) {
        const double E = F.ok ? equilibrium<D>(F, g1, g1[D - 1][z + c], x, y, -1.0 + x * h, -1.0 + y * h,
                                               -1.0 + (z + c) * h)
                              : f[c];
        q[c] = F.nup * (E - f[c]);
        o[c] = A.exact ? fma(decay, f[c] - E, E) : fma(A.dt, q[c], f[c]);
    }
    if (A.q_out) store_w<W>(A.q_out + idx, q);
    if (A.f_out) store_w<W>(A.f_out + idx, o);
}

// V rows per thread with f kept in registers: one read of f from HBM.
template <int D, int W, int V>
__global__ __launch_bounds__(kBgkThreads) void k_bgk_reg(BgkArgs A) {
    constexpr int K = D + 2;
    __shared__ double red[K * 16];
    __shared__ double S[3 * D];
    __shared__ double g1[D][512];
    const Rows<D, W> L(A.n);
    const int64_t base = (int64_t)blockIdx.x * L.rows * L.n + L.z;
    const double h = A.dv / A.T;
    double fv[V][W];
#pragma unroll
    for (int k = 0; k < V; ++k) {
        const int r = L.r0 + k * L.rstep;
        if (r < L.rows) {
            load_w<W, true>(A.f + base + (int64_t)r * L.n, fv[k]);
        } else {
#pragma unroll
            for (int c = 0; c < W; ++c) fv[k][c] = 0.0;
        }
    }
    double m[K];
#pragma unroll
    for (int a = 0; a < K; ++a) m[a] = 0.0;
    {
        int x = L.x0, y = L.y0;
#pragma unroll
        for (int k = 0; k < V; ++k) {
#pragma unroll
            for (int c = 0; c < W; ++c)   // padded rows hold 0
                add_moments<D>(m, fv[k][c], -1.0 + x * h, -1.0 + y * h, -1.0 + (L.z + c) * h);
            L.next(x, y);
        }
    }
    bgk_block_sum<K>(m, red);
    const MaxwellFit<D> F = fit_maxwellian<D>(A, m, g1, S);
    const double decay = A.exact ? exp(-F.nup * A.dt) : 0.0;
    int x = bgk_opaque(L.x0), y = bgk_opaque(L.y0);
#pragma unroll
    for (int k = 0; k < V; ++k, L.next(x, y)) {
        const int r = L.r0 + k * L.rstep;
        if (r < L.rows) emit<D, W>(A, F, g1, base + (int64_t)r * L.n, fv[k], x, y, L.z, h, decay);
    }
}

// Any cell size: f is read twice (moments, then the output pass).
template <int D, int W>
__global__ __launch_bounds__(kBgkThreads) void k_bgk(BgkArgs A) {
    constexpr int K = D + 2;
    __shared__ double red[K * 16];
    __shared__ double S[3 * D];
    __shared__ double g1[D][512];
    const Rows<D, W> L(A.n);
    const int64_t base = (int64_t)blockIdx.x * L.rows * L.n + L.z;
    const double h = A.dv / A.T;
    double m[K];
#pragma unroll
    for (int a = 0; a < K; ++a) m[a] = 0.0;
    {
        int x = L.x0, y = L.y0;
#pragma unroll FKS_BGK_UNROLL
        for (int r = L.r0; r < L.rows; r += L.rstep, L.next(x, y)) {
            double f[W];
            load_w<W, false>(A.f + base + (int64_t)r * L.n, f);
#pragma unroll
            for (int c = 0; c < W; ++c) add_moments<D>(m, f[c], -1.0 + x * h, -1.0 + y * h, -1.0 + (L.z + c) * h);
        }
    }
    bgk_block_sum<K>(m, red);
    const MaxwellFit<D> F = fit_maxwellian<D>(A, m, g1, S);
    const double decay = A.exact ? exp(-F.nup * A.dt) : 0.0;
    int x = L.x0, y = L.y0;
#pragma unroll FKS_BGK_UNROLL
    for (int r = L.r0; r < L.rows; r += L.rstep, L.next(x, y)) {
        const int64_t idx = base + (int64_t)r * L.n;
        double f[W];
        load_w<W, true>(A.f + idx, f);
        emit<D, W>(A, F, g1, idx, f, x, y, L.z, h, decay);
    }
}

// Gram matrix of (1, u_1..u_d, |u|^2), u_j = -1 + 2j/n, over the n^d grid, from
// 1D power sums, inverted in long double.
void scaled_gram_inverse(int dim, int n, double* ginv) {
    long double S[5] = {0, 0, 0, 0, 0};
    for (int j = 0; j < n; ++j) {
        long double u = -1.0L + 2.0L * j / n, p = 1.0L;
        for (int k = 0; k < 5; ++k) {
            S[k] += p;
            p *= u;
        }
    }
    const int K = dim + 2;
    const long double N1 = S[0];
    long double Nd1 = 1.0L, Nd2 = 1.0L;   // n^(d-1), n^(d-2)
    for (int a = 0; a < dim - 1; ++a) Nd1 *= N1;
    for (int a = 0; a < dim - 2; ++a) Nd2 *= N1;
    long double G[5][5] = {};
    G[0][0] = Nd1 * N1;
    for (int a = 1; a <= dim; ++a) {
        G[0][a] = G[a][0] = S[1] * Nd1;
        for (int b = 1; b <= dim; ++b) G[a][b] = (a == b) ? S[2] * Nd1 : S[1] * S[1] * Nd2;
        G[a][K - 1] = G[K - 1][a] = S[3] * Nd1 + (dim - 1) * S[1] * S[2] * Nd2;
    }
    G[0][K - 1] = G[K - 1][0] = dim * S[2] * Nd1;
    G[K - 1][K - 1] = dim * S[4] * Nd1 + dim * (dim - 1) * S[2] * S[2] * Nd2;
    long double M[5][10] = {};
    for (int a = 0; a < K; ++a) {
        for (int b = 0; b < K; ++b) M[a][b] = G[a][b];
        M[a][K + a] = 1.0L;
    }
    for (int c = 0; c < K; ++c) {
        int piv = c;
        for (int r = c + 1; r < K; ++r)
            if (fabsl(M[r][c]) > fabsl(M[piv][c])) piv = r;
        for (int k = 0; k < 2 * K; ++k) std::swap(M[c][k], M[piv][k]);
        long double d = M[c][c];
        for (int k = 0; k < 2 * K; ++k) M[c][k] /= d;
        for (int r = 0; r < K; ++r)
            if (r != c) {
                long double f = M[r][c];
                for (int k = 0; k < 2 * K; ++k) M[r][k] -= f * M[c][k];
            }
    }
    for (int a = 0; a < K; ++a)
        for (int b = 0; b < K; ++b) ginv[a * K + b] = (double)M[a][K + b];
}

}  // namespace

hipError_t bgk(const fks_bgk_desc& d, const double* f, double* q_out, double* f_out, int64_t ncell,
               double dt_over_tau, hipStream_t st) {
    BgkArgs a{};
    a.f = f;
    a.q_out = q_out;
    a.f_out = f_out;
    a.ncell = ncell;
    a.n = d.n;
    a.T = d.T;
    a.dv = 2.0 * d.T / d.n;
    a.nu = d.nu;
    a.nu_rho = d.nu_rho;
    a.exact = d.step == FKS_BGK_EXACT;
    a.dt = dt_over_tau;
    scaled_gram_inverse(d.dim, d.n, a.ginv);
    if (ncell > 0x7fffffffLL) return hipErrorInvalidValue;
    const unsigned g = (unsigned)ncell;
    const int rows = d.dim == 3 ? d.n * d.n : d.n;
    if (d.n % 2) {   // odd n: one node per access, two reads
        const int nt = d.n * (kBgkThreads / d.n);
        if (d.dim == 3) k_bgk<3, 1><<<g, nt, 0, st>>>(a);
        else k_bgk<2, 1><<<g, nt, 0, st>>>(a);
        return hipGetLastError();
    }
    const int cg = d.n / 2;
    const int nt = cg * (kBgkThreads / cg);
    const int per = (rows + nt / cg - 1) / (nt / cg);   // rows per thread
    if (d.dim == 3) {
        if (per <= 1) k_bgk_reg<3, 2, 1><<<g, nt, 0, st>>>(a);
        else if (per <= 2) k_bgk_reg<3, 2, 2><<<g, nt, 0, st>>>(a);
        else if (per <= 4) k_bgk_reg<3, 2, 4><<<g, nt, 0, st>>>(a);
        else if (per <= 8) k_bgk_reg<3, 2, 8><<<g, nt, 0, st>>>(a);
        else if (per <= 16) k_bgk_reg<3, 2, 16><<<g, nt, 0, st>>>(a);
        else if (per <= 32 && kBgkMaxRows >= 32) k_bgk_reg<3, 2, 32><<<g, nt, 0, st>>>(a);
        else k_bgk<3, 2><<<g, nt, 0, st>>>(a);
    } else {
        if (per <= 1) k_bgk_reg<2, 2, 1><<<g, nt, 0, st>>>(a);
        else if (per <= 2) k_bgk_reg<2, 2, 2><<<g, nt, 0, st>>>(a);
        else if (per <= 4) k_bgk_reg<2, 2, 4><<<g, nt, 0, st>>>(a);
        else if (per <= 8) k_bgk_reg<2, 2, 8><<<g, nt, 0, st>>>(a);
        else if (per <= 16) k_bgk_reg<2, 2, 16><<<g, nt, 0, st>>>(a);
        else if (per <= 32 && kBgkMaxRows >= 32) k_bgk_reg<2, 2, 32><<<g, nt, 0, st>>>(a);
        else k_bgk<2, 2><<<g, nt, 0, st>>>(a);
    }
    return hipGetLastError();
}

}  // namespace fks
