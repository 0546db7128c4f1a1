// Owner-map maintenance and state import/export kernels (gfx950).
//
// The owner map is kept incrementally when spheres move, in one launch with
// one wavefront per new sphere and one per old sphere, in any order:
//  - stamp: sphere c takes every node of its new ball unless a wall or a
//    lower-index sphere whose new ball also covers it owns the node; it takes
//    the node by compare-and-swap from any other owner (a higher index, the
//    fluid, or a lower index that is leaving the node);
//  - vacate: a node the previous geometry's sphere a owned and its new ball
//    does not cover turns fluid by compare-and-swap from a, if no sphere has
//    taken it, and is refilled with the equilibrium at rho0 and the velocity
//    it had as a solid (the solid-side Maxwell equilibrium of Sec. 2.3).
// Every node ends with the owner of the new geometry whatever the order of
// the workgroups: the lowest-index sphere whose new ball covers it (walls
// first), else fluid.  A node refilled and then taken by another sphere was
// refilled for nothing: a solid node's populations are never read.
#include "lbm_device.h"
#include "lbm_internal.h"

#include <hip/hip_runtime.h>
#include <math.h>

#include <algorithm>

namespace lbm {
namespace {

using namespace dev;

// A node of the lattice: wrapped coordinates and index.
struct Node {
    int px, py, pz;
    uint32_t n;
};

// Compare-and-swap of a 16-bit owner code (through its 32-bit word): the
// code found (expect on success).
__device__ __forceinline__ uint16_t cas_u16(uint16_t *addr, uint16_t expect, uint16_t val)
{
    unsigned int *w = (unsigned int *)((uintptr_t)addr & ~(uintptr_t)3);
    const unsigned int sh = ((uintptr_t)addr & 2) ? 16u : 0u;
    unsigned int old = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while (true) {
        const uint16_t cur = (uint16_t)((old >> sh) & 0xffffu);
        if (cur != expect) return cur;
        const unsigned int nw = (old & ~(0xffffu << sh)) | ((unsigned int)val << sh);
        const unsigned int prev = atomicCAS(w, old, nw);
        if (prev == old) return expect;
        old = prev;  // this code or the other half of the word changed
    }
}

// Sphere `id` (new geometry) takes node v, found with owner o.
__device__ __forceinline__ void stamp_node(const GeomArgs &g, uint16_t *own, const Node &v, uint16_t o, uint16_t id)
{
    while (true) {
        if (o < g.n_walls || o == id) return;
        if (o < id) {
            // a lower-index sphere keeps the node if its new ball covers it
            const int b = o - g.n_walls;
            if (b < g.nb2) {
                const double *Bo = g.bodies2 + (size_t)b * kBodyStride;
                if (body_ok(Bo, g.nx, g.ny, g.nz) && inside(Bo, v.px, v.py, v.pz, g.nx, g.ny, g.nz)) return;
            }
        }
        const uint16_t prev = cas_u16(own + v.n, o, id);
        if (prev == o) return;
        o = prev;
    }
}

// The nodes of ball B in the column (px, py) of the lattice: the unwrapped z
// range [lo, hi] (empty when lo > hi), exactly those for which inside() holds.
// The range is [Z - h, Z + h] with h^2 = R^2 - (dx^2 + dy^2).  A first pass
// in FP32 takes the offsets from the box origin (kx - ox for the column at
// box position kx; |offsets| <= R + 1) and bounds h^2 within +-eps2, an upper
// bound of its FP32 error with a wide margin; where both bounds give the same
// end nodes those are the ends of the exact range (the FP64 test of inside()
// differs from the exact one only within about 1e-13 of the surface).
// Otherwise the FP64 pass decides: dx^2 + dy^2 formed as inside() forms it
// and FP64 h settle every node farther than 1e-6 from both ends (their
// roundings move an end by about 2^-52 R^2 / h < 1e-7 while h > max(1e-4,
// 1e-8 R^2)), and inside() itself decides the rest: along a column |p - X|^2
// grows with |z - Z| (each rounding is monotone), so the nodes inside form
// one range.
struct BallCols {
    float ox, oy, oz;  // centre minus box origin, per axis
    float r2, eps2;    // R^2 and the error bound of h^2
    float m;           // bound of the error of a range end, with margin
};

__device__ __forceinline__ BallCols ball_cols(const double *B, const Box &bx)
{
    BallCols bc;
    bc.ox = (float)(B[0] - (double)bx.x0);
    bc.oy = (float)(B[1] - (double)bx.y0);
    bc.oz = (float)(B[2] - (double)bx.z0);
    bc.r2 = (float)(B[9] * B[9]);
    // the FP32 error of h^2 stays below 1e-6 (R + 1)^2 and that of an end
    // (the offset oz, the sums, the square root) below 1e-6 (R + 1): the
    // bounds below are ten times these
    bc.eps2 = 1e-5f * (bc.r2 + 1.0f) + 2e-5f * (float)B[9];
    bc.m = 1e-5f * ((float)B[9] + 1.0f);
    return bc;
}

__device__ __forceinline__ void column_range(const double *B, const Box &bx, const BallCols &bc, int kx, int ky,
                                             int px, int py, int nx, int ny, int nz, int &lo, int &hi)
{
#pragma clang fp contract(off)
    lo = 1;
    hi = 0;
    {
        const float dx = (float)kx - bc.ox, dy = (float)ky - bc.oy;
        const float h2 = bc.r2 - (dx * dx + dy * dy);
        if (h2 < -bc.eps2) return;  // no node of the column within R
        if (h2 > bc.eps2) {
            const float hl = __builtin_sqrtf(h2 - bc.eps2), hh = __builtin_sqrtf(h2 + bc.eps2);
            const float m = bc.m;
            // an end settled this way lies at least m / 2 from every node
            const int l0 = (int)ceilf(bc.oz - hh - m), l1 = (int)ceilf(bc.oz - hl + m);
            const int h0 = (int)floorf(bc.oz + hl - m), h1 = (int)floorf(bc.oz + hh + m);
            if (l0 == l1 && h0 == h1) {
                lo = bx.z0 + l0;
                hi = bx.z0 + h0;
                return;
            }
        }
    }
    const double r2 = B[9] * B[9];
    const double dx = min_image((double)px - B[0], nx);
    const double dy = min_image((double)py - B[1], ny);
    const double sxy = dx * dx + dy * dy;
    if (sxy > r2) return;  // |p - X|^2 >= sxy for every node of the column
    const double h = sqrt(r2 - sxy);
    const double za = B[2] - h, zb = B[2] + h;
    const double fa = floor(za), fb = floor(zb);
    lo = (int)fa + 1;
    hi = (int)fb;
    constexpr double kSure = 1e-6;
    if (h > 1e-4 && h > 1e-8 * r2 && za - fa > kSure && fa + 1.0 - za > kSure && zb - fb > kSure && fb + 1.0 - zb > kSure)
        return;
    const int zmin = (int)ceil(B[2] - B[9]), zmax = (int)floor(B[2] + B[9]);  // the ball's box
    lo = max(lo - 2, zmin);
    hi = min(hi + 1, zmax);
    while (lo <= hi && !inside(B, px, py, wrap1(lo, nz), nx, ny, nz)) ++lo;
    while (hi >= lo && !inside(B, px, py, wrap1(hi, nz), nx, ny, nz)) --hi;
}

constexpr int kColU = 8;         // nodes of a lane whose owner loads are in flight together
constexpr int kColsPerLane = 4;  // columns of a stamp lane whose nodes are taken together

__global__ __launch_bounds__(kBlock) void k_walls_init(const uint8_t *wall, uint16_t *own, int N)
{
    const int n = blockIdx.x * kBlock + threadIdx.x;
    if (n < N) own[n] = wall[n] ? (uint16_t)(wall[n] - 1) : kFluid;
}

// Lattice coordinates of node index n (a rare path: integer divisions).
__device__ __forceinline__ Node node_of(uint32_t n, int nx, int ny)
{
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny, r = n % plane;
    return Node{(int)(r % (uint32_t)nx), (int)(r / (uint32_t)nx), (int)(n / plane), n};
}

// One wavefront per job: jobs 0 .. nb2 - 1 stamp new sphere b, jobs nb2 ..
// nb2 + nb - 1 vacate old sphere b, all in any order.  The lanes take the
// (x, y) columns of the sphere's box, kColsPerLane at a time; each column's
// range of ball nodes comes from column_range, and the owner codes of a
// lane's nodes are loaded kColU at a time across its columns, so that a job
// waits for few memory round trips.
template <int S>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_geometry(GeomArgs g)
{
    using St = Store<S>;
    __shared__ uint32_t cand[kColU][kBlock];  // vacate: a lane's leaving nodes, flushed kColU at a time
    // the job is the same on every lane of the wavefront: made uniform, so that
    // its sphere records are scalar loads
    const int w = __builtin_amdgcn_readfirstlane(blockIdx.x * (kBlock / 64) + (int)(threadIdx.x >> 6));
    if (w >= g.nb + g.nb2) return;
    // stamp and vacate jobs alternate while both last (the two kinds cost
    // differently); job < nb2 stamps sphere job, else vacates job - nb2
    const int mb = min(g.nb, g.nb2);
    const int job = w < 2 * mb ? ((w & 1) ? g.nb2 + (w >> 1) : (w >> 1))
                               : (g.nb2 > g.nb ? w - mb : g.nb2 + (w - mb));
    const int lane = threadIdx.x & 63, tid = threadIdx.x;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    const uint32_t plane = (uint32_t)nx * (uint32_t)ny;
    uint16_t *own = g.own;
    if (job < g.nb2) {
        // stamp: every node of the new ball not yet owned by the sphere
        const double *B = g.bodies2 + (size_t)job * kBodyStride;
        if (!body_ok(B, nx, ny, nz)) return;
        const uint16_t id = (uint16_t)(g.n_walls + job);
        const Box bx = body_box(B, 0);
        const BallCols bc = ball_cols(B, bx);
        const int ncols = bx.ex * bx.ey;
        for (int cb = 0; cb < ncols; cb += 64 * kColsPerLane) {
            // the lane's columns: first z, node count, column index
            int lo[kColsPerLane], cum[kColsPerLane + 1];
            uint32_t cx[kColsPerLane];
            cum[0] = 0;
#pragma unroll
            for (int j = 0; j < kColsPerLane; ++j) {
                const int c = cb + j * 64 + lane;
                int l = 1, h = 0;
                cx[j] = 0;
                if (c < ncols) {
                    const int ky = c / bx.ex, kx = c - ky * bx.ex;
                    const int px = wrap1(bx.x0 + kx, nx), py = wrap1(bx.y0 + ky, ny);
                    column_range(B, bx, bc, kx, ky, px, py, nx, ny, nz, l, h);
                    cx[j] = (uint32_t)(px + nx * py);
                }
                lo[j] = l;
                cum[j + 1] = cum[j] + max(h - l + 1, 0);
            }
            // the lane's nodes k = 0 .. cum[kColsPerLane] - 1, column by column
            for (int k0 = 0; k0 < cum[kColsPerLane]; k0 += kColU) {
                uint32_t nn[kColU];
                unsigned todo = 0;
#pragma unroll
                for (int u = 0; u < kColU; ++u) {
                    const int k = k0 + u;
                    int z = lo[0] + k;
                    uint32_t col = cx[0];
#pragma unroll
                    for (int j = 1; j < kColsPerLane; ++j)
                        if (k >= cum[j]) {
                            z = lo[j] + (k - cum[j]);
                            col = cx[j];
                        }
                    nn[u] = col + plane * (uint32_t)wrap1(z, nz);
                    if (k < cum[kColsPerLane] && own[nn[u]] != id) todo |= 1u << u;
                }
                // the nodes not yet the sphere's (few: most were already)
                while (todo) {
                    const int u = __builtin_ctz(todo);
                    todo &= todo - 1;
                    uint32_t n = nn[0];
#pragma unroll
                    for (int v = 1; v < kColU; ++v)
                        if (u == v) n = nn[v];
                    stamp_node(g, own, node_of(n, nx, ny), own[n], id);
                }
            }
        }
    } else if (job < g.nb2 + g.nb) {
        // vacate: nodes of the old ball outside the new one that the sphere
        // still owns turn fluid (unless another sphere takes them first) and
        // are refilled
        const int b = job - g.nb2;
        const double *B = g.bodies + (size_t)b * kBodyStride;
        if (!body_ok(B, nx, ny, nz)) return;
        typename St::T *pop = static_cast<typename St::T *>(g.pop);
        const double *Bn = g.bodies2 + (size_t)b * kBodyStride;
        const bool keeps = b < g.nb2 && body_ok(Bn, nx, ny, nz);
        const uint16_t id = (uint16_t)(g.n_walls + b);
        const Box bx = body_box(B, 0);
        int cnt = 0;
        auto flush = [&]() {
            uint32_t nn[kColU];
            uint16_t o[kColU];
#pragma unroll
            for (int u = 0; u < kColU; ++u) {
                nn[u] = u < cnt ? cand[u][tid] : 0u;
                o[u] = u < cnt ? own[nn[u]] : (uint16_t)0;
            }
#pragma unroll
            for (int u = 0; u < kColU; ++u) {
                if (u >= cnt || o[u] != id || cas_u16(own + nn[u], id, kFluid) != id) continue;
                const Node v = node_of(nn[u], nx, ny);
                double u0, u1, u2;
                sphere_velocity(B, v.px, v.py, v.pz, nx, ny, nz, u0, u1, u2);
                for (int i = 0; i < kQ; ++i)
                    St::st(at(pop + (size_t)i * g.Ns, v.n), (float)eq_dev(i, g.rho0, u0, u1, u2));
            }
            cnt = 0;
        };
        const BallCols bc = ball_cols(B, bx);
        Box bxn{};
        BallCols bcn{};
        if (keeps) {
            bxn = body_box(Bn, 0);
            bcn = ball_cols(Bn, bxn);
        }
        for (int c = lane; c < bx.ex * bx.ey; c += 64) {
            const int ky = c / bx.ex, kx = c - ky * bx.ex;
            const int px = wrap1(bx.x0 + kx, nx), py = wrap1(bx.y0 + ky, ny);
            int lo, hi, nlo = 1, nhi = 0;
            column_range(B, bx, bc, kx, ky, px, py, nx, ny, nz, lo, hi);
            if (lo > hi) continue;
            if (keeps) {
                // the column's position in the new ball's box (the image nearest its origin)
                int kxn = px - bxn.x0, kyn = py - bxn.y0;
                if (kxn < 0) kxn += nx; else if (kxn >= nx) kxn -= nx;
                if (kyn < 0) kyn += ny; else if (kyn >= ny) kyn -= ny;
                if (kxn < bxn.ex && kyn < bxn.ey) column_range(Bn, bxn, bcn, kxn, kyn, px, py, nx, ny, nz, nlo, nhi);
            }
            // the new range as a periodic interval of wrapped z: start ns, length nlen
            const int ns = wrap1(nlo, nz), nlen = max(nhi - nlo + 1, 0);
            const uint32_t col = (uint32_t)(px + nx * py);
            for (int vz = lo; vz <= hi; ++vz) {
                const int pz = wrap1(vz, nz);
                int d = pz - ns;
                if (d < 0) d += nz;
                if (d < nlen) continue;  // stays in the ball
                cand[cnt][tid] = col + plane * (uint32_t)pz;
                if (++cnt == kColU) flush();
            }
        }
        if (cnt) flush();
    }
}

template <int S>
__global__ __launch_bounds__(kBlock) void k_init_pop(GeomArgs g, const double *rho, const double *u)
{
    using St = Store<S>;
    typename St::T *pop = static_cast<typename St::T *>(g.pop);
    const int n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.N) return;
    const size_t N = (size_t)g.N;
    if (g.own[n] < kVacated) {
        for (int i = 0; i < kQ; ++i) St::st(pop + i * (size_t)g.Ns + n, 0.0f);
        return;
    }
    const double r = rho ? rho[n] : (double)g.rho0;
    const double u0 = u ? u[n] : 0.0, u1 = u ? u[N + n] : 0.0, u2 = u ? u[2 * N + n] : 0.0;
    const double uu = u0 * u0 + u1 * u1 + u2 * u2;
    for (int i = 0; i < kQ; ++i) {
        const double cu = dcx(i) * u0 + dcy(i) * u1 + dcz(i) * u2;
        const double dev = wgt(i) * (r - (double)g.rho0) + wgt(i) * r * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
        St::st(pop + i * (size_t)g.Ns + n, (float)dev);
    }
}

__device__ __forceinline__ void solid_velocity(const GeomArgs &g, const double *walls, uint16_t o, int px, int py,
                                               int pz, double &u0, double &u1, double &u2)
{
    if (o < g.n_walls) {
        u0 = walls[o * kWallStride];
        u1 = walls[o * kWallStride + 1];
        u2 = walls[o * kWallStride + 2];
    } else {
        sphere_velocity(g.bodies + (o - g.n_walls) * kBodyStride, px, py, pz, g.nx, g.ny, g.nz, u0, u1, u2);
    }
}

template <int S>
__global__ __launch_bounds__(kBlock) void k_export_pop(GeomArgs g, const double *walls, int dir, double *out)
{
    using St = Store<S>;
    const typename St::T *pop = static_cast<const typename St::T *>(g.pop);
    const int n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.N) return;
    const uint16_t o = g.own[n];
    if (o >= kVacated) {
        out[n] = (double)St::ld(pop + (size_t)dir * g.Ns + n) + wgt(dir) * (double)g.rho0;
        return;
    }
    const int px = n % g.nx, py = (n / g.nx) % g.ny, pz = n / (g.nx * g.ny);
    double u0, u1, u2;
    solid_velocity(g, walls, o, px, py, pz, u0, u1, u2);
    out[n] = wgt(dir) * (double)g.rho0 + eq_dev(dir, g.rho0, u0, u1, u2);
}

template <int S>
__global__ __launch_bounds__(kBlock) void k_import_pop(int N, int Ns, int dir, float rho0, const double *in, void *popv)
{
    using St = Store<S>;
    typename St::T *pop = static_cast<typename St::T *>(popv);
    const int n = blockIdx.x * kBlock + threadIdx.x;
    if (n < N) St::st(pop + (size_t)dir * Ns + n, (float)(in[n] - wgt(dir) * (double)rho0));
}

template <int S>
__global__ __launch_bounds__(kBlock) void k_export_macro(GeomArgs g, const double *walls, double fx, double fy,
                                                         double fz, double *rho, double *u)
{
    using St = Store<S>;
    const typename St::T *pop = static_cast<const typename St::T *>(g.pop);
    const int n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.N) return;
    const size_t N = (size_t)g.N;
    const uint16_t o = g.own[n];
    if (o >= kVacated) {
        double r = 0.0, j0 = 0.0, j1 = 0.0, j2 = 0.0;
        for (int i = 0; i < kQ; ++i) {
            const double f = (double)St::ld(pop + i * (size_t)g.Ns + n) + wgt(i) * (double)g.rho0;
            r += f;
            j0 += dcx(i) * f;
            j1 += dcy(i) * f;
            j2 += dcz(i) * f;
        }
        rho[n] = r;
        u[n] = (j0 - 0.5 * fx) / r;
        u[N + n] = (j1 - 0.5 * fy) / r;
        u[2 * N + n] = (j2 - 0.5 * fz) / r;
        return;
    }
    const int px = n % g.nx, py = (n / g.nx) % g.ny, pz = n / (g.nx * g.ny);
    double u0, u1, u2;
    solid_velocity(g, walls, o, px, py, pz, u0, u1, u2);
    rho[n] = g.rho0;
    u[n] = u0;
    u[N + n] = u1;
    u[2 * N + n] = u2;
}

__global__ __launch_bounds__(kBlock) void k_export_owner(const uint16_t *own, int N, int32_t *out)
{
    const int n = blockIdx.x * kBlock + threadIdx.x;
    if (n < N) out[n] = own[n] >= kVacated ? -1 : (int32_t)own[n];
}

__global__ __launch_bounds__(kBlock) void k_zero(double *p, int n)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

__global__ __launch_bounds__(kBlock) void k_count_fluid(const uint16_t *own, int N, unsigned long long *count)
{
    __shared__ unsigned int s_cnt;
    if (threadIdx.x == 0) s_cnt = 0;
    __syncthreads();
    unsigned int c = 0;
    for (int n = blockIdx.x * kBlock + threadIdx.x; n < N; n += gridDim.x * kBlock) c += own[n] >= kVacated;
    atomicAdd(&s_cnt, c);
    __syncthreads();
    if (threadIdx.x == 0 && s_cnt) atomicAdd(count, (unsigned long long)s_cnt);
}

inline int nblk(long n) { return (int)((n + kBlock - 1) / kBlock); }

template <template <int> class K, typename... A>
hipError_t dispatch(int storage, dim3 grid, dim3 block, hipStream_t s, A... args)
{
    switch (storage) {
    case 0: hipLaunchKernelGGL(K<0>::fn, grid, block, 0, s, args...); break;
    case 1: hipLaunchKernelGGL(K<1>::fn, grid, block, 0, s, args...); break;
    case 2: hipLaunchKernelGGL(K<2>::fn, grid, block, 0, s, args...); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int S> struct GeomK { static constexpr auto fn = k_geometry<S>; };
template <int S> struct InitK { static constexpr auto fn = k_init_pop<S>; };
template <int S> struct ExportK { static constexpr auto fn = k_export_pop<S>; };
template <int S> struct ImportK { static constexpr auto fn = k_import_pop<S>; };
template <int S> struct MacroK { static constexpr auto fn = k_export_macro<S>; };

}  // namespace

hipError_t launch_walls_init(const uint8_t *wall, uint16_t *own, int N, hipStream_t s)
{
    hipLaunchKernelGGL(k_walls_init, dim3(nblk(N)), dim3(kBlock), 0, s, wall, own, N);
    return hipGetLastError();
}

hipError_t launch_geometry(int storage, const GeomArgs &g, hipStream_t s)
{
    const int jobs = g.nb + g.nb2;
    if (jobs <= 0) return hipSuccess;
    const int grid = (jobs + kBlock / 64 - 1) / (kBlock / 64);
    return dispatch<GeomK>(storage, dim3(grid), dim3(kBlock), s, g);
}

hipError_t launch_init_pop(int storage, const GeomArgs &g, const double *rho, const double *u, hipStream_t s)
{
    return dispatch<InitK>(storage, dim3(nblk(g.N)), dim3(kBlock), s, g, rho, u);
}

hipError_t launch_export_pop(int storage, const GeomArgs &g, const double *walls, int dir, double *out,
                             hipStream_t s)
{
    return dispatch<ExportK>(storage, dim3(nblk(g.N)), dim3(kBlock), s, g, walls, dir, out);
}

hipError_t launch_import_pop(int storage, int N, int Ns, int dir, float rho0, const double *in, void *pop,
                             hipStream_t s)
{
    return dispatch<ImportK>(storage, dim3(nblk(N)), dim3(kBlock), s, N, Ns, dir, rho0, in, pop);
}

hipError_t launch_export_macro(int storage, const GeomArgs &g, const double *walls, double fx, double fy,
                               double fz, double *rho, double *u, hipStream_t s)
{
    return dispatch<MacroK>(storage, dim3(nblk(g.N)), dim3(kBlock), s, g, walls, fx, fy, fz, rho, u);
}

hipError_t launch_export_owner(const uint16_t *own, int N, int32_t *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_export_owner, dim3(nblk(N)), dim3(kBlock), 0, s, own, N, out);
    return hipGetLastError();
}

hipError_t launch_zero(double *p, int n, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3(nblk(n)), dim3(kBlock), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_count_fluid(const uint16_t *own, int N, unsigned long long *count, hipStream_t s)
{
    hipLaunchKernelGGL(k_count_fluid, dim3(std::min(nblk(N), 2048)), dim3(kBlock), 0, s, own, N, count);
    return hipGetLastError();
}

}  // namespace lbm
