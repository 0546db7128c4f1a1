// The fused D3Q19 step on gfx950: boundary links, pull streaming, collision
// and store of a 256-node tile in one pass over HBM.
//
// Per tile (one workgroup, one node per thread):
//  1. The owner codes of the tile and of a one-node periodic halo go into
//     LDS; each thread issues the 19 pulls of its node (the streaming
//     equation of Sec. 2.2).
//  2. Each fluid node marks the directions whose pull source is a solid node
//     (a cut link, Sec. 2.3); the links of the tile are listed in LDS and
//     spread over the workgroup's threads.  Per link: the value of the
//     population the node receives (the q < 1/2 and q >= 1/2 branches with
//     the moving-boundary term of eq. moving_boundary_velocity, walls at
//     q = 1/2), formed from the current state at the node and at the node
//     behind it, which the tile's pulls have brought into the caches; and
//     the momentum exchanged on the link (Sec. 2.3, force and torque), added
//     as 64-bit fixed point to the tile's LDS table of bodies.
//  3. Each node takes its link values in place of the pulled ones, then
//     moments, the Smagorinsky relaxation time, BGK + Guo collision and the
//     store follow as in the pull-collide kernel.
//  4. The tile's body sums go to the global fixed-point sums with one atomic
//     add per body and component; a small kernel turns them into the FP64
//     forces of the step.  Integer sums do not depend on the order of the
//     additions, so the forces are the same bit for bit for every launch,
//     tile shape and batch.
// The link arithmetic is that of the boundary-link pass (lbm_linkmath.h), so
// the populations equal, bit for bit, those of the link pass followed by the
// pull-collide kernel.
#include "lbm_collide.h"
#include "lbm_device.h"
#include "lbm_internal.h"
#include "lbm_linkmath.h"

#include <hip/hip_runtime.h>
#include <math.h>

namespace lbm {
namespace {

using namespace dev;

constexpr int kLinkCap = 1024;  // links of a tile held in LDS at once (rounds beyond)
constexpr int kRec = 64;        // bodies of a tile with a slot in the LDS force table

template <int TX, int TY, int TZ>
struct FusedLds {
    static constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2, NH = HX * HY * HZ;
    uint16_t own[NH + (NH & 1)];      // owner codes of the tile and its halo, x fastest
    uint16_t item[kLinkCap];          // link: node of the tile << 5 | I
    float val[kQ - 1][kBlock];        // link value of population I at node n: val[I - 1][n]
    int key[kRec];                    // owner code of the body in a force slot, -1 free
    unsigned long long sum[kRec][6];  // fixed-point F, T of that body
    int wtot[kBlock / 64];
};

// Coordinate v >= -1 taken into [0, n).
__device__ __forceinline__ int wrap_mod(int v, int n)
{
    if (v < 0) return v + n;
    if (v < n) return v;
    return v - n < n ? v - n : v % n;
}

__device__ __forceinline__ unsigned long long to_fix(double v)
{
    return (unsigned long long)__double2ll_rn(v * kFixScale);
}

// Global fixed-point sums of owner code `key` (tile t picks the wall copy).
__device__ __forceinline__ unsigned long long *fix_slot(const FusedArgs &f, int key, int t)
{
    const int e = key < f.n_walls ? f.wall_base + key * kWallRep + (t & (kWallRep - 1)) : key - f.n_walls;
    return f.fsum + 6 * (size_t)e;
}

// Add one link's fixed-point force and torque to the tile's slot of body
// `key`, or straight to the global sums when the table is full.
template <class L>
__device__ __forceinline__ void table_add(const FusedArgs &f, L &lds, int key, const unsigned long long (&v)[6],
                                          int t)
{
    int s = key & (kRec - 1);
#pragma unroll 1
    for (int p = 0; p < kRec; ++p) {
        const int cur = atomicCAS(&lds.key[s], -1, key);
        if (cur == -1 || cur == key) {
#pragma unroll
            for (int c = 0; c < 6; ++c) atomicAdd(&lds.sum[s][c], v[c]);
            return;
        }
        s = (s + 1) & (kRec - 1);
    }
    unsigned long long *g = fix_slot(f, key, t);
#pragma unroll
    for (int c = 0; c < 6; ++c) atomicAdd(g + c, v[c]);
}

// Link j of the tile's list: its value into lds.val[j], its momentum into
// the force table.
template <int S, int TX, int TY, int TZ>
__device__ __forceinline__ void fused_link(const FusedArgs &f, FusedLds<TX, TY, TZ> &lds, int x0, int y0, int z0,
                                           int j, int t)
{
    using St = Store<S>;
    using T = typename St::T;
    using Lds = FusedLds<TX, TY, TZ>;
    constexpr int HX = Lds::HX, HY = Lds::HY;
    const StepArgs &a = f.s;
    const T *__restrict__ src = static_cast<const T *>(a.src);
    const size_t Ns = (size_t)a.Ns;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int it = lds.item[j];
    const int nl = it >> 5, I = it & 31, K = opp(I);
    const int lx = nl % TX, ly = (nl / TX) % TY, lz = nl / (TX * TY);
    const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
    const int cx = dcx(I), cy = dcy(I), cz = dcz(I);
    const int hc = ((lz + 1) * HY + (ly + 1)) * HX + lx + 1;
    const int off = cx + HX * (cy + HY * cz);
    const int os = lds.own[hc - off];  // the solid node p = x - c_I
    const uint32_t xi = (uint32_t)(x + nx * (y + ny * z));
    const float fk = St::ld(at(src + (size_t)K * Ns, xi));
    float vr;
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (os < f.n_walls) {
        const double *wl = f.walls + os * kWallStride;
        vr = St::round(fk + wall_term(wl, I, a.rho0));
        double a0, a1, a2;
        wall_arm(wl, I, x, y, z, a0, a1, a2);
        link_force(link_momentum(fk, vr, I, a.rho0), I, a0, a1, a2, acc);
    } else {
        // both second populations are loaded with the first, before q
        // decides between them
        const bool behind = lds.own[hc + off] >= kVacated;
        const float fa = St::ld(at(src + (size_t)I * Ns, xi));
        float fb = 0.0f;
        if (behind) {
            const uint32_t bi = (uint32_t)(wrap1(x + cx, nx) + nx * (wrap1(y + cy, ny) + ny * wrap1(z + cz, nz)));
            fb = St::ld(at(src + (size_t)K * Ns, bi));
        }
        const SphereK k = sphere_k(f.bodies + (size_t)(os - f.n_walls) * kBodyStride);
        const LinkGeo g = link_geo(k, f.halfway != 0, a.rho0, x, y, z, nx, ny, nz, I);
        vr = St::round(link_value(g.q, fk, fa, fb, behind, g.mw));
        double a0, a1, a2;
        sphere_arm(g, I, a0, a1, a2);
        link_force(link_momentum(fk, vr, I, a.rho0), I, a0, a1, a2, acc);
    }
    lds.val[I - 1][nl] = vr;
    unsigned long long v[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) v[c] = to_fix(acc[c]);
    table_add(f, lds, os, v, t);
}

// Tile t of the lattice of f.  Every thread of the workgroup calls it (it
// holds barriers); lds may be reused by the next call.
template <int S, int TX, int TY, int TZ>
__device__ __forceinline__ void fused_tile(const FusedArgs &f, int t, FusedLds<TX, TY, TZ> &lds)
{
    static_assert(TX * TY * TZ == kBlock, "tile must hold one workgroup");
    using St = Store<S>;
    using T = typename St::T;
    using Lds = FusedLds<TX, TY, TZ>;
    constexpr int HX = Lds::HX, HY = Lds::HY, NH = Lds::NH;
    constexpr int HU = (NH + kBlock - 1) / kBlock;
    const StepArgs &a = f.s;
    const T *__restrict__ src = static_cast<const T *>(a.src);
    T *__restrict__ dst = static_cast<T *>(a.dst);
    const size_t Ns = (size_t)a.Ns;
    const int nx = a.nx, ny = a.ny, nz = a.nz;

    const int tid = threadIdx.x;
    const int r = t / a.ntx;
    const int x0 = (t - r * a.ntx) * TX, y0 = (r % a.nty) * TY, z0 = (r / a.nty) * TZ;
    const int lx = tid % TX, ly = (tid / TX) % TY, lz = tid / (TX * TY);
    const int x = x0 + lx, y = y0 + ly, z = z0 + lz;
    const bool in = x < nx && y < ny && z < nz;
    const uint32_t idx = in ? (uint32_t)(x + nx * (y + ny * z)) : 0u;

    // 1. own code, halo codes, pulls
    const uint16_t o = in ? *at(a.own, idx) : uint16_t(0);
    uint16_t hv[HU];
#pragma unroll
    for (int u = 0; u < HU; ++u) {
        const int k = tid + u * kBlock;
        hv[u] = 0;
        if (k < NH) {
            const int hx = k % HX, hr = k / HX;
            const int gx = wrap_mod(x0 + hx - 1, nx), gy = wrap_mod(y0 + hr % HY - 1, ny);
            const int gz = wrap_mod(z0 + hr / HY - 1, nz);
            hv[u] = *at(a.own, (uint32_t)(gx + nx * (gy + ny * gz)));
        }
    }
    const bool fluid = in && o >= kVacated;
    __syncthreads();  // the previous tile's readers of lds are done
#pragma unroll
    for (int u = 0; u < HU; ++u) {
        const int k = tid + u * kBlock;
        if (k < NH) lds.own[k] = hv[u];
    }
    for (int k = tid; k < kRec; k += kBlock) lds.key[k] = -1;
    for (int k = tid; k < kRec * 6; k += kBlock) (&lds.sum[0][0])[k] = 0ull;
    if (__syncthreads_or(fluid) == 0) return;

    // 2. cut links: pull sources owned by a solid (not the inflow plane's
    //    directions from the removed domain)
    const int hc = ((lz + 1) * HY + (ly + 1)) * HX + lx + 1;
    uint32_t m = 0;
    if (fluid) {
        const bool plane = z == a.zieb_z;
#pragma unroll
        for (int i = 1; i < kQ; ++i) {
            if (CZ[i] == 1 && plane) continue;
            if (lds.own[hc - (CX[i] + HX * (CY[i] + HY * CZ[i]))] < kVacated) m |= 1u << i;
        }
    }
    int tot;
    const int pos = block_scan(__popc(m), lds.wtot, tot);
    // the link values go into LDS first; the pulls follow (the values pulled
    // across cut links are then replaced)
    for (int base = 0; base < tot; base += kLinkCap) {
        if (base) __syncthreads();  // the previous round's list is processed
        {
            int k = pos;
            uint32_t mm = m;
            while (mm) {
                const int i = __builtin_ctz(mm);
                mm &= mm - 1;
                if (k >= base && k < base + kLinkCap) lds.item[k - base] = (uint16_t)((tid << 5) | i);
                ++k;
            }
        }
        __syncthreads();
        const int n = min(kLinkCap, tot - base);
        for (int j = tid; j < n; j += kBlock) fused_link<S, TX, TY, TZ>(f, lds, x0, y0, z0, j, t);
    }
    __syncthreads();  // the link values and the tile's body sums are complete
    // 4. the tile's body sums
    if (tot > 0 && tid < kRec) {
        const int key = lds.key[tid];
        if (key >= 0) {
            unsigned long long *gs = fix_slot(f, key, t);
#pragma unroll
            for (int c = 0; c < 6; ++c) {
                const unsigned long long v = lds.sum[tid][c];
                if (v) atomicAdd(gs + c, v);
            }
        }
    }
    // 3. pull, collide and store (whole wavefronts; none with no fluid lane)
    if (!in || __ballot(fluid) == 0) return;
    float g[kQ];
    if (!fluid) {
#pragma unroll
        for (int i = 0; i < kQ; ++i) g[i] = 0.0f;
    } else {
        const int xp = x + 1 == nx ? 0 : x + 1, xm = x == 0 ? nx - 1 : x - 1;
        const int yp = y + 1 == ny ? 0 : y + 1, ym = y == 0 ? ny - 1 : y - 1;
        const int zp = z + 1 == nz ? 0 : z + 1, zm = z == 0 ? nz - 1 : z - 1;
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            const int sx = CX[i] > 0 ? xm : (CX[i] < 0 ? xp : x);
            const int sy = CY[i] > 0 ? ym : (CY[i] < 0 ? yp : y);
            const int sz = CZ[i] > 0 ? zm : (CZ[i] < 0 ? zp : z);
            g[i] = St::ld(at(src + (size_t)i * Ns, (uint32_t)(sx + nx * (sy + ny * sz))));
        }
#pragma unroll
        for (int i = 1; i < kQ; ++i)
            if ((m >> i) & 1u) g[i] = lds.val[i - 1][tid];
    }
    if (fluid && z == a.zieb_z) zieb_plane<S>(a, src, idx, g);
    collide_store<S>(a, g, fluid, idx, dst);
}

template <int S, int TX, int TY, int TZ>
__global__ __launch_bounds__(kBlock) void k_fused(FusedArgs f)
{
    __shared__ FusedLds<TX, TY, TZ> lds;
    fused_tile<S, TX, TY, TZ>(f, xcd_remap(blockIdx.x, gridDim.x), lds);
}

__global__ __launch_bounds__(kBlock) void k_finish(FinishArgs fa)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    const int ns = 6 * fa.nb;
    if (i < ns) {
        const unsigned long long v = fa.fsum[i];
        fa.fsum[i] = 0ull;
        fa.out[i] = (double)(long long)v * (1.0 / kFixScale);
    } else if (i < ns + 6 * fa.n_walls) {
        const int w = (i - ns) / 6, c = (i - ns) % 6;
        unsigned long long *p = fa.fsum + 6 * ((size_t)fa.wall_base + (size_t)w * kWallRep) + c;
        unsigned long long s = 0ull;
        for (int r = 0; r < kWallRep; ++r) {
            s += p[6 * r];
            p[6 * r] = 0ull;
        }
        fa.out[i] = (double)(long long)s * (1.0 / kFixScale);
    }
}

__global__ __launch_bounds__(kBlock) void k_zero_fix(unsigned long long *p, int n)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

// Persistent fused step over the tiles of many lattices, all with the
// batch's tile shape.  Member m owns the global tiles [tile_begin[m],
// tile_begin[m + 1]); XCD k (workgroups k, k + 8, ...) walks the k-th eighth
// of the global tile range, so that each XCD works on neighbouring tiles of
// the same members.
template <int S, int TX, int TY, int TZ>
__global__ __launch_bounds__(kBlock) void k_batch_fused(BatchStepArgs b)
{
    __shared__ FusedLds<TX, TY, TZ> lds;
    const int xcd = blockIdx.x & 7, stride = gridDim.x >> 3;
    const int lo = (int)((long long)b.total_tiles * xcd / 8), hi = (int)((long long)b.total_tiles * (xcd + 1) / 8);
    // the member of the previous tile is kept: a workgroup's next tile is
    // usually in the same member
    int mb = 0, me = 0;
    FusedArgs f{};
    for (int gt = lo + (int)(blockIdx.x >> 3); gt < hi; gt += stride) {
        if (gt < mb || gt >= me) {
            int m = 0, top = b.n;  // largest m with tile_begin[m] <= gt
            while (top - m > 1) {
                const int mid = (m + top) >> 1;
                if (b.members[mid].tile_begin <= gt) m = mid;
                else top = mid;
            }
            const BatchMember &bm = b.members[m];
            mb = bm.tile_begin;
            me = m + 1 < b.n ? b.members[m + 1].tile_begin : b.total_tiles;
            FusedArgs t = bm.f;
            const int c = b.cur[m];
            t.s.src = bm.pop[c];
            t.s.dst = bm.pop[c ^ 1];
            f = uniform(t);
        }
        fused_tile<S, TX, TY, TZ>(f, gt - mb, lds);
    }
}

// Forces of every member of a batch: one thread per force entry.
__global__ __launch_bounds__(kBlock) void k_batch_finish(BatchStepArgs b)
{
    const int g = blockIdx.x * kBlock + threadIdx.x;
    if (g >= b.total_forces) return;
    int m = 0, top = b.n;  // largest m with force_begin[m] <= g
    while (top - m > 1) {
        const int mid = (m + top) >> 1;
        if (b.members[mid].force_begin <= g) m = mid;
        else top = mid;
    }
    const FinishArgs &fa = b.members[m].fin;
    const int i = g - b.members[m].force_begin;
    const int ns = 6 * fa.nb;
    if (i < ns) {
        const unsigned long long v = fa.fsum[i];
        fa.fsum[i] = 0ull;
        fa.out[i] = (double)(long long)v * (1.0 / kFixScale);
    } else {
        const int w = (i - ns) / 6, c = (i - ns) % 6;
        unsigned long long *p = fa.fsum + 6 * ((size_t)fa.wall_base + (size_t)w * kWallRep) + c;
        unsigned long long s = 0ull;
        for (int r = 0; r < kWallRep; ++r) {
            s += p[6 * r];
            p[6 * r] = 0ull;
        }
        fa.out[i] = (double)(long long)s * (1.0 / kFixScale);
    }
}

__global__ __launch_bounds__(kBlock) void k_batch_flip(int *cur, int n)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) cur[i] ^= 1;
}

template <int S>
hipError_t launch_fused_s(const FusedArgs &f, hipStream_t s)
{
    const dim3 grid(f.s.n_tiles), block(kBlock);
    switch (f.s.tile) {
    case kTile64x2x2: hipLaunchKernelGGL((k_fused<S, 64, 2, 2>), grid, block, 0, s, f); break;
    case kTile32x4x2: hipLaunchKernelGGL((k_fused<S, 32, 4, 2>), grid, block, 0, s, f); break;
    case kTile32x2x4: hipLaunchKernelGGL((k_fused<S, 32, 2, 4>), grid, block, 0, s, f); break;
    case kTile16x8x2: hipLaunchKernelGGL((k_fused<S, 16, 8, 2>), grid, block, 0, s, f); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int S>
const void *batch_kernel_s(int shape)
{
    switch (shape) {
    case kTile64x2x2: return (const void *)k_batch_fused<S, 64, 2, 2>;
    case kTile32x4x2: return (const void *)k_batch_fused<S, 32, 4, 2>;
    case kTile32x2x4: return (const void *)k_batch_fused<S, 32, 2, 4>;
    case kTile16x8x2: return (const void *)k_batch_fused<S, 16, 8, 2>;
    default: return nullptr;
    }
}

const void *batch_kernel(int storage, int shape)
{
    switch (storage) {
    case 0: return batch_kernel_s<0>(shape);
    case 1: return batch_kernel_s<1>(shape);
    case 2: return batch_kernel_s<2>(shape);
    default: return nullptr;
    }
}

inline int nblk(long n) { return (int)((n + kBlock - 1) / kBlock); }

}  // namespace

hipError_t launch_fused(int storage, const FusedArgs &f, hipStream_t s)
{
    switch (storage) {
    case 0: return launch_fused_s<0>(f, s);
    case 1: return launch_fused_s<1>(f, s);
    case 2: return launch_fused_s<2>(f, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_finish(const FinishArgs &fa, hipStream_t s)
{
    const int n = 6 * (fa.nb + fa.n_walls);
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_finish, dim3(nblk(n)), dim3(kBlock), 0, s, fa);
    return hipGetLastError();
}

hipError_t launch_zero_fix(unsigned long long *p, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero_fix, dim3(nblk(n)), dim3(kBlock), 0, s, p, n);
    return hipGetLastError();
}

int batch_step_blocks_per_cu(int storage, int shape)
{
    const void *k = batch_kernel(storage, shape);
    int n = 0;
    if (!k || hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, k, kBlock, 0) != hipSuccess || n < 1) return 1;
    return n;
}

hipError_t launch_batch_step(int storage, int shape, const BatchStepArgs &b, int grid, hipStream_t s)
{
    if (b.total_tiles <= 0) return hipSuccess;
    const void *k = batch_kernel(storage, shape);
    if (!k) return hipErrorInvalidValue;
    BatchStepArgs arg = b;
    void *args[] = {&arg};
    return hipLaunchKernel(k, dim3(grid), dim3(kBlock), args, 0, s);
}

hipError_t launch_batch_finish(const BatchStepArgs &b, hipStream_t s)
{
    if (b.total_forces <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_batch_finish, dim3(nblk(b.total_forces)), dim3(kBlock), 0, s, b);
    return hipGetLastError();
}

hipError_t launch_batch_flip(int *cur, int n, hipStream_t s)
{
    hipLaunchKernelGGL(k_batch_flip, dim3(nblk(n)), dim3(kBlock), 0, s, cur, n);
    return hipGetLastError();
}

}  // namespace lbm
