// Owner-map maintenance and state import/export kernels (gfx950).
//
// The owner map is kept incrementally when spheres move, in one launch with
// one workgroup per new sphere and one per old sphere, in any order:
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

// Offset of box coordinate v from centre coordinate c, folded to the
// nearest periodic image in FP64 and then rounded once to FP32, so that its
// rounding error is relative to the folded offset (at most half an FP32 ulp
// of the ball's radius plus one), not to the box size.
__device__ __forceinline__ float foff(int v, double c, int n) { return (float)min_image((double)v - c, n); }

// The nodes of old ball B's box with the (8, 8, 4) workgroup, skipping those
// surely outside B and, when keeps, those surely inside the new ball Bn:
// FP32 offsets with a margin that covers their rounding (the exact FP64
// tests are left to f, which sees every node either test could accept).
template <typename F>
__device__ __forceinline__ void walk_leaving(const double *B, const double *Bn, bool keeps, int nx, int ny, int nz,
                                             int tx, int ty, int tz, F &&f)
{
    const Box bx = body_box(B, 0);
    const float R2 = (float)(B[9] * B[9]);
    const float out2 = R2 + 0.01f + 1e-5f * R2;
    const float Rn2 = keeps ? (float)(Bn[9] * Bn[9]) : 0.0f;
    const float in2 = keeps ? Rn2 - (0.01f + 1e-5f * Rn2) : -1.0f;
    const double cx = keeps ? Bn[0] : 0.0, cy = keeps ? Bn[1] : 0.0, cz = keeps ? Bn[2] : 0.0;
    for (int kz = tz; kz < bx.ez; kz += 4) {
        const int vz = bx.z0 + kz, pz = wrap1(vz, nz);
        const float dz = foff(vz, B[2], nz), ez = foff(vz, cz, nz);
        for (int ky = ty; ky < bx.ey; ky += 8) {
            const int vy = bx.y0 + ky, py = wrap1(vy, ny);
            const float dy = foff(vy, B[1], ny), ey = foff(vy, cy, ny);
            const float dyz = dy * dy + dz * dz, eyz = ey * ey + ez * ez;
            for (int kx = tx; kx < bx.ex; kx += 8) {
                const int vx = bx.x0 + kx;
                const float dx = foff(vx, B[0], nx);
                if (dx * dx + dyz > out2) continue;
                if (keeps) {
                    const float ex = foff(vx, cx, nx);
                    if (ex * ex + eyz < in2) continue;
                }
                const int px = wrap1(vx, nx);
                f(px, py, pz, px + nx * (py + ny * pz));
            }
        }
    }
}

constexpr int kBoxU = 8;  // box nodes per thread whose owner loads are in flight together

// Node k (x fastest) of a body's box: its coordinates and index.
struct BoxNode {
    int vx, vy, vz;   // unwrapped
    int px, py, pz;
    uint32_t n;
};

__device__ __forceinline__ BoxNode box_node(const Box &bx, int k, int nx, int ny, int nz)
{
    const int kx = k % bx.ex, r = k / bx.ex;
    BoxNode v;
    v.vx = bx.x0 + kx;
    v.vy = bx.y0 + r % bx.ey;
    v.vz = bx.z0 + r / bx.ey;
    v.px = wrap1(v.vx, nx);
    v.py = wrap1(v.vy, ny);
    v.pz = wrap1(v.vz, nz);
    v.n = (uint32_t)(v.px + nx * (v.py + ny * v.pz));
    return v;
}

// The nodes of a body's box in chunks of kBoxU per thread (a 1-D
// workgroup): the owner codes of a chunk are loaded together (keep(node)
// selects the nodes to load), then act(node, owner) runs on each loaded node
// whose owner passes want(owner).  Only the box index k and the node index
// are held across the loads; the coordinates are made again for act.
template <typename Keep, typename Want, typename Act>
__device__ __forceinline__ void box_chunks(const Box &bx, int nx, int ny, int nz, const uint16_t *own, Keep &&keep,
                                           Want &&want, Act &&act)
{
    const int total = bx.ex * bx.ey * bx.ez;
    for (int base = 0; base < total; base += kBoxU * kBlock) {
        uint32_t n[kBoxU];
        uint16_t o[kBoxU];
        unsigned ld = 0;
#pragma unroll
        for (int u = 0; u < kBoxU; ++u) {
            const int k = base + u * kBlock + (int)threadIdx.x;
            o[u] = 0;
            n[u] = 0;
            if (k < total) {
                const BoxNode v = box_node(bx, k, nx, ny, nz);
                if (keep(v)) {
                    ld |= 1u << u;
                    n[u] = v.n;
                    o[u] = own[v.n];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < kBoxU; ++u)
            if (((ld >> u) & 1u) && want(o[u])) act(box_node(bx, base + u * kBlock + (int)threadIdx.x, nx, ny, nz), o[u]);
    }
}

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
__device__ __forceinline__ void stamp_node(const GeomArgs &g, uint16_t *own, const BoxNode &v, uint16_t o, uint16_t id)
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

__global__ __launch_bounds__(kBlock) void k_walls_init(const uint8_t *wall, uint16_t *own, int N)
{
    const int n = blockIdx.x * kBlock + threadIdx.x;
    if (n < N) own[n] = wall[n] ? (uint16_t)(wall[n] - 1) : kFluid;
}

// Workgroups 0 .. nb2 - 1 stamp new sphere b, workgroups nb2 .. nb2 + nb - 1
// vacate old sphere b - nb2, all in any order.
template <int S>
__global__ __launch_bounds__(kBlock) void k_geometry(GeomArgs g)
{
    using St = Store<S>;
    const int tid = threadIdx.x;
    const int nx = g.nx, ny = g.ny, nz = g.nz;
    uint16_t *own = g.own;
    // stamp: nodes surely inside the new ball (FP32 with a margin that covers
    // its rounding) skip the exact FP64 test
    if ((int)blockIdx.x < g.nb2) {
        const int b = blockIdx.x;
        const double *B = g.bodies2 + (size_t)b * kBodyStride;
        if (body_ok(B, nx, ny, nz)) {
            const uint16_t id = (uint16_t)(g.n_walls + b);
            const float R2 = (float)(B[9] * B[9]), mg = 0.01f + 1e-5f * R2;
            const float in2 = R2 - mg, out2 = R2 + mg;
            box_chunks(
                body_box(B, 0), nx, ny, nz, own,
                [&](const BoxNode &v) {
                    const float dx = foff(v.vx, B[0], nx), dy = foff(v.vy, B[1], ny), dz = foff(v.vz, B[2], nz);
                    const float d2 = dx * dx + dy * dy + dz * dz;
                    if (d2 > out2) return false;
                    return d2 < in2 || inside(B, v.px, v.py, v.pz, nx, ny, nz);
                },
                [&](uint16_t o) { return o != id; }, [&](const BoxNode &v, uint16_t o) { stamp_node(g, own, v, o, id); });
        }
    } else {
        // vacate: a node the old sphere owns lies inside its old ball; one
        // surely inside the new ball stays owned
        const int b = blockIdx.x - g.nb2;
        const double *B = g.bodies + (size_t)b * kBodyStride;
        if (body_ok(B, nx, ny, nz)) {
            typename St::T *pop = static_cast<typename St::T *>(g.pop);
            const double *Bn = g.bodies2 + (size_t)b * kBodyStride;
            const bool keeps = b < g.nb2 && body_ok(Bn, nx, ny, nz);
            const uint16_t id = (uint16_t)(g.n_walls + b);
            walk_leaving(B, Bn, keeps, nx, ny, nz, tid & 7, (tid >> 3) & 7, tid >> 6, [&](int px, int py, int pz, int n) {
                if (own[n] != id || (keeps && inside(Bn, px, py, pz, nx, ny, nz))) return;
                if (cas_u16(own + n, id, kFluid) != id) return;  // taken by another sphere meanwhile
                double u0, u1, u2;
                sphere_velocity(B, px, py, pz, nx, ny, nz, u0, u1, u2);
                for (int i = 0; i < kQ; ++i) St::st(pop + (size_t)i * g.Ns + n, (float)eq_dev(i, g.rho0, u0, u1, u2));
            });
        }
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
    const int grid = g.nb + g.nb2;
    if (grid <= 0) return hipSuccess;
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
