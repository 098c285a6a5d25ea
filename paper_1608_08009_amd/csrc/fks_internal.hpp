// Internal declarations shared by the C ABI (fks_abi.hip) and the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <utility>
#include <vector>

#include "../../include/fks.h"
#include "fks_fft.hpp"

namespace fks {

// Grid constants used by the FP64 conservation step.  The invariants are taken
// in the scaled basis phi = (1, v_x/T, v_y/T, v_z/T, |v|^2/T^2); the projector
// C^T (C C^T)^{-1} C does not depend on an invertible change of basis.
struct GridConst {
    double T;         // half box
    double dv;        // grid step 2T/n
    double ginv[25];  // inverse Gram matrix of the scaled basis over the grid (row-major)
};

// The same for two velocity dimensions: basis (1, v_x/T, v_y/T, |v|^2/T^2).
struct GridConst2 {
    double T;
    double dv;
    double ginv[16];
};

// Integer velocity-index shifts of one transport step (per axis, per 1D index).
struct ShiftTable {
    int8_t s[3][64];
};

// Schedule of one (plan, ncell): fused path one workgroup per cell (1) or pairs (0),
// -1 = the cost model; multi-pass path cells per pass batch, 0 = the default.
struct Schedule {
    int one = -1;
    int chunk = 0;
    int terms = 0;   // multi-pass path: consecutive terms per launch, 0 = the default
};

}  // namespace fks

struct fks_plan {
    fks_plan_desc desc;      // with defaults resolved
    int M = 0, K = 0, J = 0; // directions, radial terms, convolution terms (M*K + 1)
    int H = 0;               // table points per term: (n/2+1) n^2 (3D), n^2 (2D)
    double kappa = 0.0;      // pi / T
    fks::GridConst gc{};
    std::vector<double> dirs;       // [M][4] (e_x, e_y, e_z, w)
    std::vector<double> rad_nodes;  // [nq]       (empty for the hard-sphere closed form)
    std::vector<double> rad_coef;   // [nq][K]
    double* d_tab64 = nullptr;      // [J][H][2] (omega*alpha, beta) FP64
    float* d_tab32 = nullptr;       // same, rounded to FP32 (FP32 plans only)
    float* d_tab32p = nullptr;      // fused kernels: d_tab32's planes kz < n/2 as
                                    // [J][n/4][n][n][2] complex (kz pairs adjacent)
    fks::GridConst* d_gc = nullptr; // device copy of gc
    int dim = 3;                    // velocity dimension
    unsigned long long* d_guard = nullptr;   // first non-finite cell (numeric guard), ~0 = none
    fks::GridConst2* d_gc2 = nullptr;   // device grid constants of a dim = 2 plan
    size_t table_bytes = 0;
    bool fused = false;             // fks_collide_batch uses the fused kernel
    int fused_grid = 0;             // persistent grid of the fused kernel
    float* d_tab48p = nullptr;      // FP32 de-aliased plans at n = 32: d_tab32 zero-padded to the
                                    // 48-point grid in the layout of the n = 48 kernel's tables
    int grid48 = 0;                 // resident grid of the n = 48 kernel (those plans)
    double flops_per_cell = 0.0;
    int device = 0;
    std::vector<std::pair<int64_t, fks::Schedule>> tuned;   // measured by fks_autotune, per ncell
    int queue_ipw = 0;              // work queues led by this plan: items per resident workgroup
                                    // (0: the cost model's 4); kept by fks_autotune
};

namespace fks {

// the measured schedule of (plan, ncell), or the default Schedule{} if none
inline Schedule schedule_for(const fks_plan* p, int64_t ncell) {
    for (const auto& e : p->tuned)
        if (e.first == ncell) return e.second;
    return Schedule{};
}

// host math (fks_abi.hip)
void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w);
int radial_expansion(double gamma, double R, int K, double tol, int nq, std::vector<double>& nodes,
                     std::vector<double>& coef);
bool supported_n(int n);

// tables (fks_tables.hip)
hipError_t build_tables(fks_plan* plan, hipStream_t stream);

// multi-pass path, FP64 and FP32 (fks_generic.hip)
size_t generic_workspace_bytes(const fks_plan* plan, int64_t ncell);
bool generic_multi_terms(const fks_plan* plan);   // several terms per launch available
hipError_t collide_generic(const fks_plan* plan, const fks_segment& seg, void* ws, size_t ws_bytes,
                           hipStream_t stream);

// n = 48 FP32 forward transform for the on-chip terms kernel (fks_generic.hip): f into the
// half spectrum, [C] slots of (n/2+1) n^2 complex with the planes kz < n/2 in the kz-pair
// layout of d_tab32p (work: [C][n^3] complex)
hipError_t forward_f32_48(const double* f, cx<float>* work, cx<float>* fh, int C, hipStream_t st);
// FP32 de-aliased plans at n = 32: fill d_tab48p from d_tab32 (fks_generic.hip)
hipError_t embed_tables48(const fks_plan* p, hipStream_t st);

// n = 48 FP32 terms, three workgroups per cell (fks_fused48.hip): resident grid, and the
// launch over consecutive cell ranges (pieces) that each share a plan's tables (item
// counters [8] in device memory, cleared by the call)
constexpr int kMaxPieces48 = 16;
struct Piece48 {
    const cx<float>* tab;   // [J][n/4][n][n][2] balanced FP32 tables (d_tab32p, kz pairs adjacent)
    int64_t cell0;          // first cell of the piece in the launch's cell order
    int J;
};
// FP64 fix and update after the terms kernel, all pieces of a chunk in one launch: the
// piece's outputs are indexed by c0 + (cell - cell0)
struct Fin48 {
    const double* f_base;
    double* q_out;
    double* f_out;
    const GridConst* gc;
    unsigned long long* guard;
    double dt;
    int64_t cell0;          // first cell of the piece in the chunk
    int64_t c0;             // its first cell within its segment
};
hipError_t finish48(const float* acc, const Fin48* pieces, int npieces, int64_t ncell, hipStream_t st);
int terms48_grid(int device);
hipError_t terms48(const cx<float>* fh, const Piece48* pieces, int npieces, float* acc, int64_t ncell, int* ctr,
                   int grid, hipStream_t st);

// spectrum of a batch (multi-pass FP64, fks_generic.hip)
size_t spectrum_workspace_bytes(int n, int64_t ncell);
hipError_t spectrum(const double* x, double* xhat, int64_t ncell, int n, int zero_nyquist, void* ws, size_t ws_bytes,
                    hipStream_t st);

// optional event timing of the fused path (fks_fused.hip)
void profile_enable(bool on);
hipError_t profile_last(double* ms, int cap, int* count);

// fused single-kernel FP32 path (fks_fused.hip)
bool fused_available(int n);
int fused_grid_size(int n, int device);
size_t fused_workspace_bytes(const fks_plan* plan, int64_t ncell);
hipError_t collide_fused(const fks_plan* plan, const fks_segment& seg, void* ws, size_t ws_bytes,
                         hipStream_t stream);

// several fused segments of one n in one work queue (fks_fused.hip): at most
// fused_queue_max_segments() segments, all with ncell > 0 and the same n
int fused_queue_max_segments();
size_t fused_queue_workspace_bytes(const fks_segment* const* segs, int nseg);
hipError_t collide_fused_queue(const fks_segment* const* segs, int nseg, void* ws, size_t ws_bytes,
                               hipStream_t stream);

// two velocity dimensions (fks_2d.hip)
bool supported_n_2d(int n, int precision);
GridConst2 grid_const2(int n, double T);
void tables_2d(const fks_plan_desc& d, std::vector<double>& ab);   // [J][n][n][2]
hipError_t collide_2d(const fks_plan* plan, const fks_segment& seg, hipStream_t stream);

// BGK relaxation (fks_bgk.hip)
hipError_t bgk(const fks_bgk_desc& d, const double* f, double* q_out, double* f_out, int64_t ncell,
               double dt_over_tau, hipStream_t stream);

// moments, projection, transport (fks_aux.hip)
GridConst grid_const(int n, double T);
hipError_t moments(const double* f, int64_t ncell, int n, double T, double* U, hipStream_t stream);
hipError_t conserve(double* f, const double* U, int64_t ncell, int n, double T, hipStream_t stream);
// from_below == nullptr: the whole grid, z by sp.bc[2].  Otherwise one z slab: source planes
// -1 and nz are the messages from the neighbours below (v_z > 0) and above (v_z < 0), laid
// out as halo_pack writes them; the host has checked that the z shift stays within them
hipError_t transport(const double* f_in, double* f_out, const fks_space_desc& sp, int n,
                     const ShiftTable& shift, const double* bc_f, hipStream_t stream, const double* from_below,
                     const double* from_above);
// copies the kz range [k0, k0 + h) of every velocity row of one plane of f to buf
// [ncell_plane][n][n][h]
hipError_t halo_pack(const double* f, double* buf, int64_t plane, int64_t ncell_plane, int n, int k0, int h,
                     hipStream_t stream);

}  // namespace fks
