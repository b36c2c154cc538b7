// Internal declarations shared by the kernels (lbm_kernels.hip) and the host
// side of the C ABI (lbm_api.hip).  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>

namespace lbm {

// Population storage of one lattice, per time level: nodes are numbered
// idx = y * pitch + x (x fastest; pitch = nx in FP64 and in lattices that runs
// can step, else nx rounded up to 16 in FP32) and grouped in blocks of kBlock consecutive indices, so a block may
// hold the end of one row and the start of the next; a block holds the 27
// populations (f_0..8, g_0..8, h_0..8) as 27 runs of kBlock values.  A level
// is 27 * `plane` elements, plane = pitch * ny rounded up to whole blocks.  Levels A/B alternate every step.  f and h are stored
// as deviations from the rest equilibrium w_i phi0 and w_i T0; g as is.
constexpr int kPlanes = 27;
constexpr int kBlock = 64;
constexpr int kF = 0, kG = 9, kH = 18;
// Entries of a side's wall-temperature table before its point s = 0.
constexpr int kTwPad = 4;
// Element index, within a level, of population q of node idx.
__host__ __device__ constexpr long long pop_index(int q, long long idx)
{
    return ((idx / kBlock) * kPlanes + q) * kBlock + idx % kBlock;
}

// Per-lattice constants, in the working precision.  Properties are stored as
// xi(phi) = xi_a + xi_b * phi (linear interpolation between phi = -1 and +1).
template <typename real>
struct Inst {
    real* pop[2];        // time levels A and B
    real* jprev;         // 2 planes: (phi u)_x, (phi u)_y of the previous level
    // Address of population q of node 0 of each level (pop[l] + q * kBlock;
    // node idx adds its block offset) and the bases of the two (phi u) planes:
    // the step kernel reads them as uniform values.
    real* qbase[2][27];
    real* jbase[2];
    int nx, ny, pitch, grad_mode;
    int collision;       // 0: BGK; 1: two relaxation times for g and h
    int force_form;      // 0: mu_phi grad phi (Eq. 11); 1: -phi grad mu_phi
    real trt_magic;      // (tau+ - 1/2)(tau- - 1/2)
    long long plane;
    int bc[4];
    real phi0, T0;
    real rho_a, rho_b, mu_a, mu_b, lam_a, lam_b, rcp_a, rcp_b;
    real sigma_ref, sigma_T, sigma_TT, dTref;   // dTref = T0 - T_ref
    real W2, pref, inv_W2, inv_s2W;             // W^2, 3 sqrt(2) W / 4, 1/W^2, 1/(sqrt(2) W)
    real inv_tau_phi, fac_phi;                  // 1/tau_phi, 1 - 1/(2 tau_phi)
    real Gx, Gy;
    // Wall temperatures relative to T0 at the points s = j/2 - kTwPad/2 along
    // each side (nodes and the half-way points between them), j = 0 ..
    // tw_stride - 1, side after side: tabulated on the host at init
    const real* twall;
    int tw_stride;
    real u_in, phi_in_d, T_in_d;                // phi_in - phi0, T_in - T0
};

struct Tile {
    int inst, x0, y0, flags;
};
// Neither the tile nor its one-node ring crosses a wall, inlet or outlet:
// streaming and ring loads need at most one periodic wrap.
constexpr int kTileInterior = 1;
// The tile lies inside the lattice (else its last columns or rows do not).
constexpr int kTileWhole = 2;
// The entry is a run: TX * TY consecutive nodes in x-fastest order from node
// number x0 (y0 unused).  Interior runs hold no node of the first or last row.
constexpr int kTileRun = 4;

// Sums accumulated by the FP64 diagnostics reduction, per lattice.
enum DiagSlot {
    D_MASS = 0, D_VOL, D_HEAT, D_SNEG, D_SUY, D_SUX, D_SX, D_SY, D_MAXU, D_NONFIN, D_NNEG,
    D_BUB = 11,  // 4 regions x (sum, sum x, sum y, sum ux, sum uy)
    D_COUNT = 31
};

struct DiagArgs {
    double bx[4], by[4];
    double rcp_a, rcp_b;
    int n_bubbles;
};

struct InitArgs {
    double phi0, T0, rho_a, rho_b;
    int has_p;  // staged pressure plane present (else p = 0, or the current p when shifting)
    int shift;  // add eq(new) - eq(current fields in staged planes 5..9) instead of replacing
};

// Compiled tile shapes (TX x TY nodes, one work-item per node).  Ids from
// kTileRuns on step lattices periodic in x with kRunMinNx <= nx <= kRunMaxNx
// in runs of TX * TY consecutive nodes (rows of any width then leave no
// work-item idle) and the other lattices in their TX x TY tiles; they are not
// used with the potential form of the capillary force (those lattices take
// tiles).
constexpr int kTileCount = 8;
constexpr int kTileTX[kTileCount] = {64, 128, 32, 64, 256, 128, 128, 64};
constexpr int kTileTY[kTileCount] = {4, 2, 8, 8, 1, 4, 4, 4};
constexpr int kTileRuns = 6;
constexpr int kRunMinNx = 64, kRunMaxNx = 256;
// Nodes per run of tile id (0: not a run id).
constexpr int run_nodes(int id) { return id >= kTileRuns ? kTileTX[id] * kTileTY[id] : 0; }
// Tile id whose TX x TY table serves the field and diagnostics kernels.
constexpr int grid_tile(int id) { return id == 6 ? 5 : (id == 7 ? 0 : id); }

// Launchers (lbm_kernels.hip).  `src` is the time level read (0 = A, 1 = B).
// `variant` selects the step kernel: 0 BGK only; 1 BGK or two relaxation
// times per lattice; 2 also the potential form of the capillary force.
hipError_t launch_step(int prec, int tile, const void* insts, const Tile* tiles, int ntiles, int grid, int src,
                       int variant, hipStream_t s);
// Macroscopic fields of level `src`: any output may be null; out_f32 selects
// float outputs.  If `jprev_out` is set, (phi u) is written to the lattice's
// jprev planes instead.
hipError_t launch_fields(int prec, int tile, const void* insts, const Tile* tiles, int ntiles, int src,
                         void* phi, void* ux, void* uy, void* T, void* p, int out_f32, int jprev_out,
                         hipStream_t s);
// Equilibrium populations of one lattice from staged FP64 fields phi, ux, uy,
// T (n_nodes each, x fastest, contiguous) into time level `src`.
hipError_t launch_init(int prec, const void* inst_dev, long long n_nodes, const double* staged, const InitArgs& a,
                       int src, hipStream_t s);
// Device fields (FP32 if in_f32, else FP64) into the FP64 staging layout of launch_init.
hipError_t launch_stage(const void* phi, const void* ux, const void* uy, const void* T, const void* p, int in_f32,
                        long long n,
                        double* staged, hipStream_t s);
// Per-workgroup FP64 partial sums (D_COUNT each) then a deterministic final sum
// into `result` (D_COUNT doubles).
hipError_t launch_diag(int prec, int tile, const void* insts, const Tile* tiles, int ntiles, int src,
                       const DiagArgs& a, double* partials, double* result, hipStream_t s);

// Resident workgroups of the step kernel per compute unit.
hipError_t step_occupancy(int prec, int tile, int variant, int* blocks_per_cu);

// Plain 16-byte-vector copy of `bytes` (a multiple of 16).
hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s);

}  // namespace lbm
