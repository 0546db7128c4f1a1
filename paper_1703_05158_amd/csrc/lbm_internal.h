// Internal interface between the C-ABI host layer (lbm_api.cpp) and the
// gfx950 kernels (lbm_step.hip, lbm_links.hip, lbm_geometry.hip).  Not part
// of the ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbm {

constexpr int kQ = 19;

// Owner map codes (uint16 per node).  Solid owners are ids below kVacated:
// walls 0..n_walls-1, then spheres n_walls + b; kFluid marks the fluid
// nodes.  Every code from kVacated up counts as fluid.
constexpr uint16_t kFluid = 0xFFFF;
constexpr uint16_t kVacated = 0x8000;
constexpr int kMaxIds = 0x7FFE;

constexpr int kBodyStride = 10;   // X[3], V[3], Omega[3], R
constexpr int kWallStride = 6;    // U[3], ref[3]
constexpr int kMaxWalls = 16;
constexpr int kBlock = 256;       // threads of a workgroup
constexpr int kWallChunk = 1024;  // wall links per workgroup of the link pass

// Tile shapes of the step kernel (256 nodes, one per thread).
enum TileShape { kTile64x2x2 = 0, kTile32x4x2 = 1, kTile32x2x4 = 2, kTile16x8x2 = 3, kNumTileShapes = 4 };
constexpr int kTileDims[kNumTileShapes][3] = {{64, 2, 2}, {32, 4, 2}, {32, 2, 4}, {16, 8, 2}};

// Pull-collide step over the fluid nodes.  The populations pulled across a
// cut link come from the solid node's slot, where the link pass has put the
// bounce-back value.
struct StepArgs {
    int nx, ny, nz, N;
    int Ns;                       // stride between direction arrays (elements, >= N)
    int tile;                     // TileShape
    int ntx, nty, ntz, n_tiles;
    float tau0, smag_k, rho0;     // smag_k = 18 sqrt(2) C^2
    float fx, fy, fz;
    const uint16_t *own;
    const void *src;
    void *dst;
    int *flag;                    // NaN guard, may be null
    int zieb_z;                   // z of the inflow plane fed by a virtual cylinder, -1 = none
    const double *zieb_state;     // ZiebState: rho is the cylinder density of this step
    // wall totals of the link pass that preceded this step: workgroup w <
    // n_wsum adds the chunk sums of wall w into wsum_out[6 (wsum_nb + w)]
    int n_wsum, wsum_nb;
    const double *wsum_part;      // [chunks][6]
    const int *wsum_wblk;         // [n_walls + 1]: each wall's range of chunks
    double *wsum_out;
};

// Zoom-in with Effective Boundaries (Sec. 2.6): the state of the virtual
// cylinder below the plane z = z.
struct ZiebState {
    double rho;                   // cylinder density (< 0: take the plane's mean at the first step)
    double H;                     // piston displacement
    double vf;                    // mean inflow velocity used by the last update
    double pad;
};

constexpr int kZiebMaxBlocks = 1024;  // workgroups of the plane reduction (a grid-stride loop beyond)

struct ZiebArgs {
    int nx, ny, nz, N, Ns, z;
    float rho0, fz;
    double area, volume, vp;
    const uint16_t *own;
    const void *pop;              // current state
    double *state;                // ZiebState
    double *part;                 // [kZiebMaxBlocks][3]: per-workgroup sums
    unsigned int *done;           // workgroups finished (0 between updates)
};

// Boundary-link pass: for every link from a fluid node x to a solid node
// x + c_K, the value of the population I = opposite(K) that x receives is
// written to slot I of the solid node, and the momentum exchanged on the
// link is reduced per body.
struct LinkArgs {
    int nx, ny, nz, Ns;
    int n_walls, nb, halfway;
    float rho0;
    const uint16_t *own;
    void *pop;                    // current state: read at fluid nodes, written at solid nodes
    const double *bodies;         // [nb][kBodyStride]
    const double *walls;          // [n_walls][kWallStride]
    const double *wrec;           // [n_walls][kBodyStride]: each wall as a record {ref, U, 0, 0} for the link arithmetic
    const uint32_t *wl_node;      // fluid nodes of the wall links, grouped by (wall, direction)
    const int *wl_blk;            // [n_wblk][3]: segment w * 18 + I - 1, begin, end
    int n_wblk;
    double *wl_part;              // [n_wblk][6]
    const int *wl_wblk;           // [n_walls + 1]: each wall's range of workgroups
    double *out;                  // [nb + n_walls][6]: F, T
    const int *order;             // [nb]: the order in which spheres are taken (spatially sorted), or null
};

// Fixed-point force sums of the fused step: every link's force and torque is
// rounded to a multiple of 2^-32 and added as a 64-bit integer, so that the
// sums do not depend on the order of the additions.  Wall sums are spread
// over kWallRep copies (by tile) to keep the atomics of the many tiles that
// touch a wall off one address.
constexpr double kFixScale = 4294967296.0;  // 2^32
constexpr int kWallRep = 64;

// Turn the fixed-point sums into the FP64 forces of the step (spheres, then
// walls) and clear them for the next step.
struct FinishArgs {
    unsigned long long *fsum;
    int wall_base, nb, n_walls;
    double *out;                  // [nb + n_walls][6]
    double *out2;                 // a second copy (the caller's device buffer), or null
};

// The fused step: per tile, the boundary links of its fluid nodes (the Sec.
// 2.3 value of every population pulled across a cut link, formed from the
// current state, and the momentum exchanged on the link), then the pull,
// collision and store of the step kernel.
struct FusedArgs {
    StepArgs s;                   // the step (its wall-total fields unused)
    int n_walls, nb, halfway;
    const double *bodies;         // [nb][kBodyStride], the current geometry
    const double *wrec;           // [n_walls][kBodyStride]: each wall as a record {ref, U, 0, 0}
    unsigned long long *fsum;     // fixed-point sums: [max_bodies][6], then [n_walls][kWallRep][6]
    int wall_base;                // max_bodies: first wall copy of fsum
    FinishArgs fin;               // the previous step's sums (another buffer) to finish first, if fin.fsum
};

// One lattice of a batch: its fused-step arguments for the batch's tile
// shape (src/dst filled in per step from pop[cur]), its force finish, and
// the first global tile and force entry it owns.
struct BatchMember {
    FusedArgs f;
    FinishArgs fin;
    void *pop[2];
    int tile_begin;               // global tile index of the member's tile 0
    int force_begin;              // global index of the member's first force entry (6 per body and wall)
};

// Tile queues of the batched step: one counter per XCD, kQueueStride ints
// apart (separate cache lines), zero before each step.
constexpr int kQueueStride = 32;
constexpr int kQueueInts = 8 * kQueueStride;

struct BatchStepArgs {
    const BatchMember *members;
    const int *cur;               // [n]: member m's state is in pop[cur[m]]
    int *queue;                   // [kQueueInts]: the XCDs' next tile counters
    int n;
    int total_tiles;
    int total_forces;
};

// Reverse-mode step for the gradient of the summed sphere drag (FP32
// storage, fixed spheres, no walls).
struct AdjStepArgs {
    StepArgs a;                   // src = the state P_{n-1} the step starts from
    const float *lam;             // adjoint of the post-collision state P_n, [19][Ns]
    float *lam_prev;              // adjoint of P_{n-1}, [19][Ns]: every entry is written (see k_adj_collide)
    double *dF_tile;              // [n_tiles][3], accumulated over the steps
};

struct AdjLinkArgs {
    LinkArgs a;                   // geometry and bodies; pop unused
    const float *mu;              // adjoint of f_n at the links, in the solid slots (p, I) of a
                                  // [19][Ns] array; null: the objective's own derivative
    float *lam;                   // adjoint of P_{n-1}, links add into it
    double *dV;                   // [nb][3], accumulated over the steps
};

struct GeomArgs {
    int nx, ny, nz;
    int N;
    int Ns;                       // stride between direction arrays
    int n_walls;
    const double *bodies;         // the current (old) geometry's table, nb spheres
    int nb;
    const double *bodies2;        // the new geometry's table, nb2 spheres
    int nb2;
    uint16_t *own;
    void *pop;
    float rho0;
};

// storage: 0 = fp32, 1 = fp16, 2 = bf16 deviations
hipError_t launch_step(int storage, const StepArgs &a, hipStream_t s);
hipError_t launch_links(int storage, const LinkArgs &a, hipStream_t s);
// With start or stop events, the launch records the kernel's own start and
// end in them (no separate event packets on the stream).
hipError_t launch_fused(int storage, const FusedArgs &f, hipStream_t s, hipEvent_t start = nullptr,
                        hipEvent_t stop = nullptr);
hipError_t launch_finish(const FinishArgs &fa, hipStream_t s);
hipError_t launch_zero_fix(unsigned long long *p, int n, hipStream_t s);

// Fixed-point force sums of lbm_step_noalloc: a file-scope device array of
// two halves of kStaticFixHalf entries (1 MiB in all), shared by every call
// on a device.  static_fix_scratch gives its address on the current device
// (looked up once per device).
constexpr int kStaticFixHalf = 65536;
hipError_t static_fix_scratch(unsigned long long **out);
hipError_t launch_batch_step(int storage, int shape, const BatchStepArgs &b, int grid, hipStream_t s);
int batch_step_blocks_per_cu(int storage, int shape);   // resident workgroups per CU of the persistent step kernel
hipError_t launch_batch_finish(const BatchStepArgs &b, hipStream_t s);
hipError_t launch_batch_flip(int *cur, int n, int *queue, hipStream_t s);

hipError_t launch_zieb_update(int storage, const ZiebArgs &z, hipStream_t s);
hipError_t launch_adj_collide(const AdjStepArgs &g, hipStream_t s);
hipError_t launch_adj_links(const AdjLinkArgs &g, hipStream_t s);
hipError_t launch_adj_reduce(const double *dF_tile, int n_tiles, double *dF, hipStream_t s);

hipError_t launch_walls_init(const uint8_t *wall, uint16_t *own, int N, hipStream_t s);
hipError_t launch_geometry(int storage, const GeomArgs &g, hipStream_t s);
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
