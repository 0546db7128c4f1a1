// Boundary-link pass on gfx950: interpolated bounce-back on moving spheres,
// halfway bounce-back on moving voxel walls, and momentum exchange.
//
// For every link from a fluid node x to a solid node x + c_K (K = opposite(I))
// the value of the population I that x receives in this step (Sec. 2.3: the
// q < 1/2 and q >= 1/2 branches and eq. moving_boundary_velocity) is written
// into slot I of the solid node, in the current population buffer; the step
// kernel then pulls it like any other population.  Populations are read only
// at fluid nodes and written only at solid nodes, so workgroups never touch
// each other's data.  The momentum handed to the body along c_K (Sec. 2.3,
// force and torque equations) is reduced per body in a fixed order:
//  - one workgroup per sphere walks the sphere's box and lists candidate
//    links from the geometry alone (FP32 distances with a margin, no memory
//    access), spreads them evenly over its threads, confirms each with the
//    owner map (loads issued together with the population loads, so a link
//    costs one memory round trip) and reduces force and torque itself;
//  - wall links do not change while the walls stay: their fluid nodes are
//    listed once per (wall, direction); workgroups take chunks of the list
//    and write per-chunk sums that k_wall_forces adds up per wall.
#include "lbm_device.h"
#include "lbm_internal.h"

#include <hip/hip_runtime.h>
#include <math.h>

namespace lbm {
namespace {

using namespace dev;

constexpr int kWaves = kBlock / 64;

// Sum of NV values over the workgroup, in a fixed order; the result is valid
// in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double (*s_red)[6])
{
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int c = 0; c < NV; ++c) v[c] += __shfl_xor(v[c], off);
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int c = 0; c < NV; ++c) s_red[wv][c] = v[c];
    __syncthreads();
    if (threadIdx.x == 0)
#pragma unroll
        for (int c = 0; c < NV; ++c) {
            double t = s_red[0][c];
            for (int w = 1; w < kWaves; ++w) t += s_red[w][c];
            v[c] = t;
        }
}

// Candidate link from the fluid node x = p + c_I to the node p of sphere B
// (owner code ob): a link when p belongs to the sphere and x is fluid.
template <int S>
__device__ __forceinline__ void sphere_link(const LinkArgs &a, typename Store<S>::T *pop, const double *B,
                                            uint16_t ob, int px, int py, int pz, int I, double (&acc)[6])
{
    using St = Store<S>;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const size_t Ns = (size_t)a.Ns;
    const int K = opp(I);
    const int cx = dcx(I), cy = dcy(I), cz = dcz(I);  // c_I = -c_K
    const int x = wrap1(px + cx, nx), y = wrap1(py + cy, ny), z = wrap1(pz + cz, nz);
    const uint32_t pi = (uint32_t)(px + nx * (py + ny * pz));
    const uint32_t xi = (uint32_t)(x + nx * (y + ny * z));
    const uint32_t bi = (uint32_t)(wrap1(x + cx, nx) + nx * (wrap1(y + cy, ny) + ny * wrap1(z + cz, nz)));
    // All issued together.  Populations read at a node that turns out to be
    // solid are discarded (the load may see a link value being written there).
    const uint16_t op = *at(a.own, pi), ox = *at(a.own, xi), obk = *at(a.own, bi);
    const float fk = St::ld(at(pop + (size_t)K * Ns, xi));
    const float fi = St::ld(at(pop + (size_t)I * Ns, xi));
    const float gb = St::ld(at(pop + (size_t)K * Ns, bi));
    if (op != ob || ox < kVacated) return;
    const bool back_fluid = obk >= kVacated;

    const double ckx = -cx, cky = -cy, ckz = -cz;
    const double d0 = min_image((double)x - B[0], nx);
    const double d1 = min_image((double)y - B[1], ny);
    const double d2 = min_image((double)z - B[2], nz);
    double q;
    if (a.halfway) {
        q = 0.5;
    } else {
        // smallest root in (0,1] of |d + q c_K|^2 = R^2, cancellation-free form
        const double bb = d0 * ckx + d1 * cky + d2 * ckz;
        const double aa = (double)(cx * cx + cy * cy + cz * cz);
        const double cc = __dadd_rn(__dadd_rn(__dmul_rn(d0, d0), __dmul_rn(d1, d1)), __dmul_rn(d2, d2)) -
                          __dmul_rn(B[9], B[9]);
        const double disc = fmax(bb * bb - aa * cc, 0.0);
        q = fmin(fmax(cc / (sqrt(disc) - bb), 0.0), 1.0);
    }
    // wall point x_b = x + q c_K relative to the centre, and its velocity
    const double ar0 = d0 + q * ckx, ar1 = d1 + q * cky, ar2 = d2 + q * ckz;
    const double u0 = B[3] + (B[7] * ar2 - B[8] * ar1);
    const double u1 = B[4] + (B[8] * ar0 - B[6] * ar2);
    const double u2 = B[5] + (B[6] * ar1 - B[7] * ar0);
    // moving-boundary term along the reflected direction I
    const float wk = (float)wgt(K);
    const float mw = wk * a.rho0 * (float)(cx * u0 + cy * u1 + cz * u2);
    const float qf = (float)q;
    float val;
    if (q < 0.5) {
        val = back_fluid ? 2.0f * qf * fk + (1.0f - 2.0f * qf) * gb + 6.0f * mw : fk + 6.0f * mw;
    } else {
        const float h = 0.5f / qf;
        val = h * fk + (1.0f - h) * fi + (3.0f / qf) * mw;
    }
    const float vr = St::round(val);
    St::st(at(pop + (size_t)I * Ns, pi), vr);
    // momentum handed to the body along c_K (full populations)
    const double mom = (double)fk + (double)vr + 2.0 * (double)wk * (double)a.rho0;
    const double F0 = mom * ckx, F1 = mom * cky, F2 = mom * ckz;
    acc[0] += F0;
    acc[1] += F1;
    acc[2] += F2;
    acc[3] += ar1 * F2 - ar2 * F1;
    acc[4] += ar2 * F0 - ar0 * F2;
    acc[5] += ar0 * F1 - ar1 * F0;
}

struct SphereLds {
    uint16_t item[kBlock * (kQ - 1)];  // candidate links of one round: node slot | I << 8
    int px[kBlock], py[kBlock], pz[kBlock];
    int wtot[kWaves];
};

// Sphere b, in rounds of one box node per thread.  A node p is a candidate
// when its FP32 distance to the centre is within a margin of the ball and
// more than R - 1.5 (deeper nodes have no neighbour outside), and (p, I) is
// a candidate link when p + c_I lies outside the ball by the same margin.
// The margin covers the FP32 rounding, so every link is a candidate; the
// owner map then decides exactly.
template <int S>
__device__ __forceinline__ void sphere_block(const LinkArgs &a, int b, SphereLds &L, double (*s_red)[6])
{
    using St = Store<S>;
    typename St::T *pop = static_cast<typename St::T *>(a.pop);
    const double *B = a.bodies + (size_t)b * kBodyStride;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (body_ok(B, nx, ny, nz)) {
        const Box bx = body_box(B, 0);
        const int total = bx.ex * bx.ey * bx.ez;
        const uint16_t ob = (uint16_t)(a.n_walls + b);
        const float R2 = (float)(B[9] * B[9]);
        const float mg = 0.01f + 1e-5f * R2;
        const float ri = (float)B[9] - 1.5f;
        const float in2 = ri > 0.0f ? ri * ri - mg : -1.0f;
        for (int base = 0; base < total; base += kBlock) {
            const int k = base + tid;
            uint32_t lm = 0;
            if (k < total) {
                const int kx = k % bx.ex, kr = k / bx.ex;
                const int px = wrap1(bx.x0 + kx, nx), py = wrap1(bx.y0 + kr % bx.ey, ny),
                          pz = wrap1(bx.z0 + kr / bx.ey, nz);
                L.px[tid] = px;
                L.py[tid] = py;
                L.pz[tid] = pz;
                const float dx = (float)min_image((double)px - B[0], nx);
                const float dy = (float)min_image((double)py - B[1], ny);
                const float dz = (float)min_image((double)pz - B[2], nz);
                const float d2 = dx * dx + dy * dy + dz * dz;
                if (d2 <= R2 + mg && d2 >= in2) {
#pragma unroll
                    for (int i = 1; i < kQ; ++i) {
                        const float ex = dx + CX[i], ey = dy + CY[i], ez = dz + CZ[i];
                        if (ex * ex + ey * ey + ez * ez > R2 - mg) lm |= 1u << i;
                    }
                }
            }
            // exclusive scan of the candidate counts over the workgroup
            const int cnt = __popc(lm);
            int incl = cnt;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int v = __shfl_up(incl, off);
                if (lane >= off) incl += v;
            }
            if (lane == 63) L.wtot[wv] = incl;
            __syncthreads();
            int pos = incl - cnt, tot = 0;
#pragma unroll
            for (int w = 0; w < kWaves; ++w) {
                const int t = L.wtot[w];
                if (w < wv) pos += t;
                tot += t;
            }
            while (lm) {
                const int I = __builtin_ctz(lm);
                lm &= lm - 1;
                L.item[pos++] = (uint16_t)(tid | (I << 8));
            }
            __syncthreads();
#pragma unroll 1
            for (int j = tid; j < tot; j += kBlock) {
                const int it = L.item[j], sl = it & 255;
                sphere_link<S>(a, pop, B, ob, L.px[sl], L.py[sl], L.pz[sl], it >> 8, acc);
            }
            __syncthreads();  // item, px/py/pz and wtot are reused by the next round
        }
    }
    block_sum<6>(acc, s_red);
    if (tid == 0)
#pragma unroll
        for (int c = 0; c < 6; ++c) a.out[6 * b + c] = acc[c];
}

// One chunk of the links of wall w in direction I: halfway bounce-back with
// the wall velocity, q = 1/2.
template <int S>
__device__ __forceinline__ void wall_block(const LinkArgs &a, int blk, double (*s_red)[6])
{
    using St = Store<S>;
    typename St::T *pop = static_cast<typename St::T *>(a.pop);
    const int nx = a.nx, ny = a.ny;
    const size_t Ns = (size_t)a.Ns;
    const int seg = a.wl_blk[3 * blk], beg = a.wl_blk[3 * blk + 1], end = a.wl_blk[3 * blk + 2];
    const int w = seg / (kQ - 1), I = seg - (kQ - 1) * w + 1, K = opp(I);
    const int cx = dcx(I), cy = dcy(I), cz = dcz(I);  // c_I = -c_K
    const double *wl = a.walls + w * kWallStride;
    const float wk = (float)wgt(K);
    const float add = 6.0f * (wk * a.rho0 * (float)(cx * wl[0] + cy * wl[1] + cz * wl[2]));
    const double w2 = 2.0 * (double)wk * (double)a.rho0;
    // momentum sum and its first moment about the reference point; the
    // chunk's kWallChunk / kBlock links per thread have their loads in flight
    // together
    constexpr int U = kWallChunk / kBlock;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    uint32_t xi[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int j = beg + (int)threadIdx.x + u * kBlock;
        xi[u] = j < end ? a.wl_node[j] : 0xFFFFFFFFu;
    }
    uint16_t o[U];
    float fk[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
        o[u] = 0;
        fk[u] = 0.0f;
        if (xi[u] != 0xFFFFFFFFu) {
            o[u] = *at(a.own, xi[u]);
            fk[u] = St::ld(at(pop + (size_t)K * Ns, xi[u]));
        }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        if (o[u] < kVacated) continue;  // past the chunk's end, or covered by a sphere
        const uint32_t x = xi[u] % (uint32_t)nx, r = xi[u] / (uint32_t)nx;
        const uint32_t y = r % (uint32_t)ny, z = r / (uint32_t)ny;
        const int sx = wrap1((int)x - cx, nx), sy = wrap1((int)y - cy, ny), sz = wrap1((int)z - cz, a.nz);
        const float vr = St::round(fk[u] + add);
        St::st(at(pop + (size_t)I * Ns, (uint32_t)(sx + nx * (sy + ny * sz))), vr);
        const double mom = (double)fk[u] + (double)vr + w2;
        v[0] += mom;
        v[1] += mom * ((double)x - 0.5 * cx - wl[3]);
        v[2] += mom * ((double)y - 0.5 * cy - wl[4]);
        v[3] += mom * ((double)z - 0.5 * cz - wl[5]);
    }
    block_sum<4>(v, s_red);
    if (threadIdx.x == 0) {
        // F = S c_K, T = (sum mom arm) x c_K, c_K = -c_I
        double *o = a.wl_part + 6 * (size_t)blk;
        o[0] = -v[0] * cx;
        o[1] = -v[0] * cy;
        o[2] = -v[0] * cz;
        o[3] = -(v[2] * cz - v[3] * cy);
        o[4] = -(v[3] * cx - v[1] * cz);
        o[5] = -(v[1] * cy - v[2] * cx);
    }
}

template <int S>
__global__ __launch_bounds__(kBlock) void k_links(LinkArgs a)
{
    __shared__ SphereLds L;
    __shared__ double s_red[kWaves][6];
    if ((int)blockIdx.x < a.nb)
        sphere_block<S>(a, blockIdx.x, L, s_red);
    else
        wall_block<S>(a, blockIdx.x - a.nb, s_red);
}

// Wall w: the sum of its chunks' partial forces and torques.
__global__ __launch_bounds__(64) void k_wall_forces(LinkArgs a)
{
    const int w = blockIdx.x, lane = threadIdx.x;
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int j = a.wl_wblk[w] + lane; j < a.wl_wblk[w + 1]; j += 64)
#pragma unroll
        for (int c = 0; c < 6; ++c) v[c] += a.wl_part[6 * (size_t)j + c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int c = 0; c < 6; ++c) v[c] += __shfl_xor(v[c], off);
    if (lane < 6) a.out[6 * (a.nb + w) + lane] = v[lane];
}

}  // namespace

hipError_t launch_links(int storage, const LinkArgs &a, hipStream_t s)
{
    const int grid = a.nb + a.n_wblk;
    if (grid <= 0) return hipSuccess;
    switch (storage) {
    case 0: hipLaunchKernelGGL(k_links<0>, dim3(grid), dim3(kBlock), 0, s, a); break;
    case 1: hipLaunchKernelGGL(k_links<1>, dim3(grid), dim3(kBlock), 0, s, a); break;
    case 2: hipLaunchKernelGGL(k_links<2>, dim3(grid), dim3(kBlock), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_wall_forces(const LinkArgs &a, hipStream_t s)
{
    if (a.n_walls <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_wall_forces, dim3(a.n_walls), dim3(64), 0, s, a);
    return hipGetLastError();
}

}  // namespace lbm
