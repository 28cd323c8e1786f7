// kernels.h -- launch interface between the C ABI glue and the gfx950 kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace lbm {

// Launch geometry shared by every per-cell kernel.  A wavefront owns a
// 64-cell segment of one x-row; a 256-thread block owns 4 consecutive
// segments in (z, y, segment) order.  Blocks are remapped so that each of
// the 8 XCDs (which receive hardware block ids round-robin) works on one
// contiguous eighth of the domain, keeping neighbouring rows in one L2.
struct Geo {
  int32_t nx, ny, nz;
  int32_t xs;       // x stride of a population row, in cells
  uint32_t plane;   // elements from one direction array to the next (nz * ny * xs + padding)
  int32_t nseg;     // 64-cell segments per row
  int32_t nrows;    // ny * nz
  int32_t nblocks;  // blocks launched (4 segments each)
  int32_t nb8;      // nblocks rounded down to a multiple of 8
  int32_t yb;       // step kernel: rows are visited in bands of yb rows of y, z fastest
};

// Launch geometry of the two-step kernel: 64 x TY tiles in (x, y), z chunks.
struct Geo2 {
  int32_t nx, ny, nz;
  int32_t xs;      // x stride of a population row, in cells
  uint32_t plane;  // elements from one direction array to the next
  int32_t ntx, nty, zc, nblocks, nb8;
};

constexpr int kBlock = 256;
constexpr int kReduceBlocks = 1024;

struct PhysParams {
  double omega;      // 1 / tau (0 for tau = +inf)
  double F[3];       // body-force density
  double scale;      // FP16 storage scale 2^s (1 otherwise)
  double wall_u[3];  // velocity of the moving-wall cells
  bool moving;       // wall_u != 0 and the grid has flags: moving-wall markers are in use
  bool incomp;       // He-Luo incompressible equilibrium (u = j + F/2)
  bool split;        // bounce-back by the separate obstacle kernel (the paper's split design)
};

Geo make_geo(int nx, int ny, int nz, int xs, uint64_t dir_stride);

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_init(int storage, const Geo& g, const PhysParams& ph, void* grid,
                       const uint8_t* flags, const float* rho0, const float* u0, hipStream_t s);
hipError_t launch_mark_solids(int storage, const Geo& g, const PhysParams& ph, void* grid,
                              const uint8_t* flags, hipStream_t s);
hipError_t launch_step(int storage, bool solids, bool force, const Geo& g, const PhysParams& ph,
                       const void* src, void* dst, const uint8_t* flags, hipStream_t s);
// Two fused steps src = f*(t) -> dst = f*(t+2) (bit-identical to two launch_step calls;
// not for the split design).
// lmask: the link mask of launch_link_mask, or NULL (resting walls then use
// the markers; moving walls always do).
hipError_t launch_step2(int storage, bool solids, bool force, const Geo& g, const PhysParams& ph,
                        const void* src, void* dst, const uint8_t* flags, const uint32_t* lmask,
                        hipStream_t s);
// Blocks a two-step launch has on this grid (its tiles and z chunks).
int step2_blocks(int storage, const Geo& g);
// Fewer blocks than this leave most CUs idle: single steps are faster there
// (measured on periodic cubes: 112 blocks at 100^3 ran 22.0k MLUPS FP32
// against 27.5k for single steps, 160 at 128^3 40.9k against 34.2k).
constexpr int kStep2MinBlocks = 128;
// The same two steps storing the intermediate level too: mid = f*(t+1)
// (FP32 storage only: hipErrorInvalidValue otherwise).
hipError_t launch_step2_mid(int storage, bool solids, bool force, const Geo& g,
                            const PhysParams& ph, const void* src, void* mid, void* dst,
                            const uint8_t* flags, const uint32_t* lmask, hipStream_t s);
// The two-step kernel's link mask of every cell ([nz][ny][nx] uint32) from the
// flags: bit i (1..18) for a blocked pull along c_i, bits 19 and 20 for the
// cell's own SOLID and NOFORCE flags.
hipError_t launch_link_mask(const Geo& g, const uint8_t* flags, uint32_t* mask, hipStream_t s);
hipError_t launch_obstacle(int storage, const Geo& g, const PhysParams& ph, void* grid,
                           const uint8_t* flags, hipStream_t s);
hipError_t launch_macro(int storage, bool out_f64, const Geo& g, const PhysParams& ph,
                        const void* grid, const uint8_t* flags, void* rho, void* u, hipStream_t s);
hipError_t launch_reduce(int storage, const Geo& g, const PhysParams& ph, const void* grid,
                         const uint8_t* flags, double* scratch, double* out5, hipStream_t s);
// Discrete adjoint in pull form (nu = dL/df, the pre-collision adjoint):
// seed nu^T from dL/drho_T, dL/du_T and f*(T-1); step nu^{n+1} -> nu^n with
// f*(n-1); init dL/du0 from nu^1.
hipError_t launch_adj_seed(bool solids, const Geo& g, const PhysParams& ph, const float* fprev,
                           const uint8_t* flags, const float* dL_drho, const float* dL_du,
                           float* nu_T, double* partials, hipStream_t s);
hipError_t launch_adj_step(bool solids, const Geo& g, const PhysParams& ph, const float* fprev,
                           const uint8_t* flags, const float* nu_np1, float* nu_n,
                           double* partials, hipStream_t s);
hipError_t launch_adj_init(bool solids, const Geo& g, const PhysParams& ph, const uint8_t* flags,
                           const float* nu1, const float* rho0, const float* u0, float* dL_du0,
                           hipStream_t s);
hipError_t launch_adj_finish(const Geo& g, const double* partials, double* out3, hipStream_t s);
hipError_t launch_copy(void* c, const void* a, size_t n16, hipStream_t s);
// Copy variants for the bandwidth sweep: vec in {1, 2, 4} 16-byte elements per
// thread, non-temporal or not, `blocks` blocks (0 = one pass over the array).
hipError_t launch_copy_variant(void* c, const void* a, size_t n16, int vec, bool nt, size_t blocks,
                               hipStream_t s);
// Pull-copy probe: one pure-streaming pass dst_i(x) = src_i(x - c_i) (periodic,
// no geometry, no collision) with the step kernel's launch and access pattern.
hipError_t launch_pull_copy(int storage, const Geo& g, const void* src, void* dst, hipStream_t s);

}  // namespace lbm
