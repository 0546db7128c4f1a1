// Internal interface between the C-ABI host layer (lbm_api.cpp) and the
// gfx950 kernels (lbm_step.hip, lbm_geometry.hip).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int kQ = 19;

// Owner map codes (uint16 per node).  Solid owners are ids below kVacated:
// walls 0..n_walls-1, then spheres n_walls + b.  kVacated | id marks a node
// that the previous geometry's sphere `id` covered while the map is being
// rebuilt.  kNear marks fluid nodes with at least one solid neighbour among
// the 18 links; kFluid marks the remaining fluid nodes.  For kNear nodes a
// separate uint32 per node holds the solid-link mask: bit i set when the
// pull source x - c_i is solid.
constexpr uint16_t kFluid = 0xFFFF;
constexpr uint16_t kNear = 0xFFFE;
constexpr uint16_t kVacated = 0x8000;
constexpr int kMaxIds = 0x7FFE;

constexpr int kBodyStride = 10;   // X[3], V[3], Omega[3], R
constexpr int kWallStride = 6;    // U[3], ref[3]
constexpr int kMaxWalls = 16;     // walls get dedicated per-tile force slots
constexpr int kRec = 32;          // per-tile force records of spheres
constexpr int kBlock = 256;       // threads of a step workgroup (one tile)

// Tile shapes of the step kernel (x extent; y and z fill 256 threads).
enum TileShape { kTile64x2x2 = 0, kTile32x4x2 = 1 };

struct StepArgs {
    int nx, ny, nz, N;
    int Ns;                       // stride between direction arrays (elements, >= N)
    int tile;                     // TileShape
    int ntx, nty, ntz, n_tiles;
    float tau0, smag_k, rho0;     // smag_k = 18 sqrt(2) C^2
    float fx, fy, fz;
    int n_walls, nb, halfway;
    const uint16_t *own;
    const uint32_t *nmask;        // solid-link mask of near-boundary nodes
    const void *src;
    void *dst;
    const double *bodies;
    const double *walls;
    int *rec_n;                   // [n_tiles]
    int *rec_id;                  // [n_tiles][kRec]
    double *rec_v;                // [n_tiles][kRec][6]
    double *wallpart;             // [n_tiles][n_walls][6]
    double *overflow;             // [max_bodies][6], zero between steps
    double *out;                  // [nb + n_walls][6]
    int *flag;
};

struct GeomArgs {
    int nx, ny, nz;
    int N;
    int Ns;                       // stride between direction arrays
    int n_walls;
    const double *bodies;
    int nb;
    const double *bodies2;        // new geometry's table (settle pass)
    int nb2;
    uint16_t *own;
    uint32_t *nmask;
    void *pop;
    float rho0;
};

// storage: 0 = fp32, 1 = fp16, 2 = bf16 deviations
hipError_t launch_step(int storage, const StepArgs &a, hipStream_t s);
hipError_t launch_forces(const StepArgs &a, hipStream_t s);

hipError_t launch_walls_init(const uint8_t *wall, uint16_t *own, int N, hipStream_t s);
hipError_t launch_flags_full(const GeomArgs &g, hipStream_t s);
hipError_t launch_vacate(const GeomArgs &g, hipStream_t s);
hipError_t launch_stamp(const GeomArgs &g, hipStream_t s);
hipError_t launch_settle(int storage, const GeomArgs &g, hipStream_t s);
hipError_t launch_init_pop(int storage, const GeomArgs &g, const double *rho, const double *u,
                           hipStream_t s);
hipError_t launch_export_pop(int storage, const GeomArgs &g, const double *walls, int dir,
                             double *out, hipStream_t s);
hipError_t launch_import_pop(int storage, int N, int Ns, int dir, float rho0, const double *in, void *pop,
                             hipStream_t s);
hipError_t launch_export_macro(int storage, const GeomArgs &g, const double *walls, double fx,
                               double fy, double fz, double *rho, double *u, hipStream_t s);
hipError_t launch_export_owner(const uint16_t *own, int N, int32_t *out, hipStream_t s);
hipError_t launch_zero(double *p, int n, hipStream_t s);
hipError_t launch_count_fluid(const uint16_t *own, int N, unsigned long long *count,
                              hipStream_t s);

}  // namespace lbm
