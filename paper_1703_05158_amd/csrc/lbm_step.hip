// One D3Q19 step on gfx950: the pull-collide kernel.
//
// k_step computes, for every fluid node of a 256-node tile, in one pass over
// HBM: pull streaming (the streaming equation of Sec. 2.2), moments (eqs.
// dens, momentum, with the Guo half-force velocity shift), the Smagorinsky
// relaxation time of Sec. 2.2, BGK collision with the Guo source (eq.
// Collision_step), store.  A population pulled across a cut link comes from
// the solid node's slot, where the link pass of the same step has put the
// bounce-back value (Sec. 2.3).
//
// Wavefronts of solid nodes only are skipped.  In a wavefront that holds
// fluid nodes, the solid lanes store zeros in the same store instructions
// as the fluid lanes: a store with lanes switched off writes partial
// 128-byte lines, which cost a read-modify-write in HBM (one solid node per
// 64-node row made the whole step a quarter slower).  The value a solid node
// holds is never read before the link pass of the next step replaces it.
#include "lbm_collide.h"
#include "lbm_device.h"
#include "lbm_internal.h"

#include <hip/hip_runtime.h>
#include <math.h>

namespace lbm {
namespace {

using namespace dev;

// Tile t (TX x TY x TZ nodes, one per thread) of the lattice described by a.
template <int S, int TX, int TY, int TZ>
__device__ __forceinline__ void tile_step(const StepArgs &a, int t)
{
    static_assert(TX * TY * TZ == kBlock, "tile must hold one workgroup");
    using St = Store<S>;
    using T = typename St::T;
    const T *__restrict__ src = static_cast<const T *>(a.src);
    T *__restrict__ dst = static_cast<T *>(a.dst);
    const size_t Ns = (size_t)a.Ns;
    const int nx = a.nx, ny = a.ny, nz = a.nz;

    const int tid = threadIdx.x;
    const int r = t / a.ntx;
    const int x = (t - r * a.ntx) * TX + tid % TX;
    const int y = (r % a.nty) * TY + (tid / TX) % TY;
    const int z = (r / a.nty) * TZ + tid / (TX * TY);
    if (x >= nx || y >= ny || z >= nz) return;
    const uint32_t idx = (uint32_t)(x + nx * (y + ny * z));
    const bool fluid = *at(a.own, idx) >= kVacated;
    if (__ballot(fluid) == 0) return;

    // pull: population i arrives from x - c_i
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
        if (z == a.zieb_z) zieb_plane<S>(a, src, idx, g);
    }
    collide_store<S>(a, g, fluid, idx, dst);
}

// Force and torque on wall w: the sum of its link-pass chunks, by the first
// wavefront of a workgroup (lanes take every 64th chunk, then a fixed
// butterfly), so the result does not depend on the launch.
__device__ __forceinline__ void wall_total(const StepArgs &a, int w)
{
    const int lane = threadIdx.x;
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    for (int j = a.wsum_wblk[w] + lane; j < a.wsum_wblk[w + 1]; j += 64)
#pragma unroll
        for (int c = 0; c < 6; ++c) v[c] += a.wsum_part[6 * (size_t)j + c];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int c = 0; c < 6; ++c) v[c] += __shfl_xor(v[c], off);
    if (lane < 6) a.wsum_out[6 * (a.wsum_nb + w) + lane] = v[lane];
}

template <int S, int TX, int TY, int TZ>
__global__ __launch_bounds__(kBlock) void k_step(StepArgs a)
{
    if (threadIdx.x < 64)
        for (int w = blockIdx.x; w < a.n_wsum; w += gridDim.x) wall_total(a, w);
    tile_step<S, TX, TY, TZ>(a, xcd_remap(blockIdx.x, gridDim.x));
}

template <int S>
hipError_t launch_step_s(const StepArgs &a, hipStream_t s)
{
    switch (a.tile) {
    case kTile64x2x2: hipLaunchKernelGGL((k_step<S, 64, 2, 2>), dim3(a.n_tiles), dim3(kBlock), 0, s, a); break;
    case kTile32x4x2: hipLaunchKernelGGL((k_step<S, 32, 4, 2>), dim3(a.n_tiles), dim3(kBlock), 0, s, a); break;
    case kTile32x2x4: hipLaunchKernelGGL((k_step<S, 32, 2, 4>), dim3(a.n_tiles), dim3(kBlock), 0, s, a); break;
    case kTile16x8x2: hipLaunchKernelGGL((k_step<S, 16, 8, 2>), dim3(a.n_tiles), dim3(kBlock), 0, s, a); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// The virtual cylinder's update of one step: the mean in-flowing velocity
// v_f and density of the plane's fluid nodes from the current state
// (u = (sum f c - F/2)/rho), then eq. (ZIEBdesity8) for the cylinder
// density, which the plane takes in this step, and the piston displacement.
// Each workgroup sums a run of the plane in FP64; the last one to finish
// adds the workgroups' sums in workgroup order (so the result does not
// depend on the launch's timing), updates the state and clears the counter.
template <int S>
__global__ __launch_bounds__(kBlock) void k_zieb_update(ZiebArgs z)
{
    using St = Store<S>;
    const typename St::T *pop = static_cast<const typename St::T *>(z.pop);
    constexpr int kW = kBlock / 64;
    __shared__ double s_red[3][kW];
    double su = 0.0, sr = 0.0, sc = 0.0;
    const int plane = z.nx * z.ny;
    for (int k = blockIdx.x * kBlock + threadIdx.x; k < plane; k += gridDim.x * kBlock) {
        const uint32_t n = (uint32_t)(k + plane * z.z);
        if (z.own[n] < kVacated) continue;
        double rd = 0.0, jz = 0.0;
        for (int i = 0; i < kQ; ++i) {
            const double gi = (double)St::ld(pop + (size_t)i * z.Ns + n);
            rd += gi;
            jz += dcz(i) * gi;
        }
        const double r = (double)z.rho0 + rd;
        su += (jz - 0.5 * (double)z.fz) / r;
        sr += r;
        sc += 1.0;
    }
    for (int off = 32; off > 0; off >>= 1) {
        su += __shfl_xor(su, off);
        sr += __shfl_xor(sr, off);
        sc += __shfl_xor(sc, off);
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
        s_red[0][wv] = su;
        s_red[1][wv] = sr;
        s_red[2][wv] = sc;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    double bu = 0.0, br = 0.0, bc = 0.0;
    for (int w = 0; w < kW; ++w) {
        bu += s_red[0][w];
        br += s_red[1][w];
        bc += s_red[2][w];
    }
    double *pp = z.part + 3 * (size_t)blockIdx.x;
    __hip_atomic_store(pp, bu, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(pp + 1, br, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __hip_atomic_store(pp + 2, bc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    // the sums are visible before the count that announces them
    if (__hip_atomic_fetch_add(z.done, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) != gridDim.x - 1) return;
    double tu = 0.0, tr = 0.0, tc = 0.0;
    for (int b = 0; b < (int)gridDim.x; ++b) {
        const double *q = z.part + 3 * (size_t)b;
        tu += __hip_atomic_load(q, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        tr += __hip_atomic_load(q + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        tc += __hip_atomic_load(q + 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    const double vf = tc > 0.0 ? tu / tc : 0.0;
    double *st = z.state;
    const double rho = st[0] < 0.0 ? (tc > 0.0 ? tr / tc : (double)z.rho0) : st[0];
    st[0] = rho * exp((z.vp * z.area - vf * z.area) / (z.volume - z.area * st[1]));
    st[1] += z.vp;
    st[2] = vf;
    __hip_atomic_store(z.done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ---- reverse mode (gradient of the summed sphere drag) ------------------
//
// For a step P_n = C(f_n), f_n = S(P_{n-1}), k_adj_collide turns the adjoint
// lambda_n of P_n into the adjoint mu_n of the streamed populations f_n,
// mu = (dC/df)^T lambda, node by node, and adds lambda . dC/dF (the body
// force) to per-tile sums.  It applies the transpose of plain streaming in
// the same pass: f_n(x)[i] came from P_{n-1}(x - c_i)[i], so mu(x)[i] is
// pushed to lambda_{n-1}(x - c_i)[i].  Streaming is a permutation, so every
// entry of lambda_{n-1} is written once: solid nodes push zeros (nothing was
// pulled from them), and where x - c_i is solid the pushed value is the
// adjoint of a link value, which the link kernel then takes from that solid
// slot and adds to the populations the link was formed from.  The collision is recomputed from f_n:
// moments, the equilibrium, Pi, Q = Pi:Pi, tau* and the Guo source, as in
// the forward step (Sec. 2.2); the derivative of sqrt(Q) is taken as
// 1/(2 sqrt(Q + 1e-30)), finite where Q = 0.

// mu = (dC/df)^T lam at one node (deviations g = f - w rho0), and the body-
// force part added to Fb.
__device__ __forceinline__ void collide_adjoint(const StepArgs &a, const float (&g)[kQ], const float (&lam)[kQ],
                                                float (&mu)[kQ], double (&Fb)[3])
{
    const float F[3] = {a.fx, a.fy, a.fz};
    float rd = 0.f, j[3] = {0.f, 0.f, 0.f}, S[3][3] = {{0.f}};
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const int c[3] = {CX[i], CY[i], CZ[i]};
        rd += g[i];
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            j[p] += c[p] * g[i];
#pragma unroll
            for (int q = 0; q < 3; ++q)
                if (c[p] * c[q]) S[p][q] += c[p] * c[q] * g[i];
        }
    }
    const float rho = a.rho0 + rd, ir = 1.0f / rho;
    float u[3];
#pragma unroll
    for (int p = 0; p < 3; ++p) u[p] = (j[p] + 0.5f * F[p]) * ir;
    const float uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const float uF = u[0] * F[0] + u[1] * F[1] + u[2] * F[2];
    float Pi[3][3], Q = 0.f;
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            Pi[p][q] = S[p][q] - (p == q ? rd * (1.0f / 3.0f) : 0.f) - rho * u[p] * u[q];
            Q += Pi[p][q] * Pi[p][q];
        }
    const float s = __builtin_amdgcn_sqrtf(Q);  // the step's tau* takes the hardware square roots too
    const float Rr = a.tau0 * a.tau0 + a.smag_k * s * ir, sR = __builtin_amdgcn_sqrtf(Rr);
    const float om = 2.0f / (a.tau0 + sR);
    // adjoints of omega and of the equilibrium / source terms
    float Ob = 0.f;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const float w = (float)wgt(i);
        const float cu = CX[i] * u[0] + CY[i] * u[1] + CZ[i] * u[2];
        const float cF = CX[i] * F[0] + CY[i] * F[1] + CZ[i] * F[2];
        const float geq = w * (rd + rho * (3.0f * cu + 4.5f * cu * cu - 1.5f * uu));
        const float src = w * (3.0f * (cF - uF) + 9.0f * cu * cF);
        Ob += lam[i] * (-(g[i] - geq) - 0.5f * src);
    }
    const float tb = -Ob * om * om;
    const float Rb = tb * 0.25f / sR;
    float rhob = -Rb * a.smag_k * s * ir * ir;
    const float Qb = Rb * a.smag_k * ir * 0.5f / sqrtf(Q + 1e-30f);
    float Pb[3][3];
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q) Pb[p][q] = 2.0f * Pi[p][q] * Qb;
    float rdb = -(Pb[0][0] + Pb[1][1] + Pb[2][2]) * (1.0f / 3.0f);
    float ub[3] = {0.f, 0.f, 0.f};
    double fb[3] = {0.0, 0.0, 0.0};
    const float cs = 1.0f - 0.5f * om;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const int c[3] = {CX[i], CY[i], CZ[i]};
        const float w = (float)wgt(i);
        const float cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
        const float cF = c[0] * F[0] + c[1] * F[1] + c[2] * F[2];
        const float gq = om * lam[i] * w;   // adjoint of geq_i, times w_i
        const float sq = cs * lam[i] * w;   // adjoint of the source S_i, times w_i
        rdb += gq;
        rhob += gq * (3.0f * cu + 4.5f * cu * cu - 1.5f * uu);
#pragma unroll
        for (int p = 0; p < 3; ++p) {
            ub[p] += gq * rho * (3.0f * c[p] + 9.0f * cu * c[p] - 3.0f * u[p]) + sq * (-3.0f * F[p] + 9.0f * c[p] * cF);
            fb[p] += (double)(sq * (3.0f * (c[p] - u[p]) + 9.0f * cu * c[p]));
        }
    }
#pragma unroll
    for (int p = 0; p < 3; ++p)
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            rhob -= Pb[p][q] * u[p] * u[q];
            ub[p] -= 2.0f * rho * Pb[p][q] * u[q];
        }
    float jb[3];
#pragma unroll
    for (int p = 0; p < 3; ++p) {
        jb[p] = ub[p] * ir;
        rhob -= ub[p] * u[p] * ir;
        Fb[p] += fb[p] + (double)(0.5f * ub[p] * ir);
    }
    rdb += rhob;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const int c[3] = {CX[i], CY[i], CZ[i]};
        float m = (1.0f - om) * lam[i] + rdb + jb[0] * c[0] + jb[1] * c[1] + jb[2] * c[2];
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int q = 0; q < 3; ++q)
                if (c[p] * c[q]) m += Pb[p][q] * c[p] * c[q];
        mu[i] = m;
    }
}

template <int TX, int TY, int TZ>
__global__ __launch_bounds__(kBlock) void k_adj_collide(AdjStepArgs ga)
{
    const StepArgs &a = ga.a;
    const float *__restrict__ src = static_cast<const float *>(a.src);
    const size_t Ns = (size_t)a.Ns;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const int tid = threadIdx.x;
    const int t = xcd_remap(blockIdx.x, gridDim.x);
    const int r = t / a.ntx;
    const int x = (t - r * a.ntx) * TX + tid % TX;
    const int y = (r % a.nty) * TY + (tid / TX) % TY;
    const int z = (r / a.nty) * TZ + tid / (TX * TY);
    const bool in = x < nx && y < ny && z < nz;
    const uint32_t idx = in ? (uint32_t)(x + nx * (y + ny * z)) : 0u;
    const bool fluid = in && *at(a.own, idx) >= kVacated;
    double Fb[3] = {0.0, 0.0, 0.0};
    if (fluid) {
        float g[kQ], lam[kQ], mu[kQ];
        const int xp = x + 1 == nx ? 0 : x + 1, xm = x == 0 ? nx - 1 : x - 1;
        const int yp = y + 1 == ny ? 0 : y + 1, ym = y == 0 ? ny - 1 : y - 1;
        const int zp = z + 1 == nz ? 0 : z + 1, zm = z == 0 ? nz - 1 : z - 1;
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            const int sx = CX[i] > 0 ? xm : (CX[i] < 0 ? xp : x);
            const int sy = CY[i] > 0 ? ym : (CY[i] < 0 ? yp : y);
            const int sz = CZ[i] > 0 ? zm : (CZ[i] < 0 ? zp : z);
            g[i] = *at(src + (size_t)i * Ns, (uint32_t)(sx + nx * (sy + ny * sz)));
            lam[i] = *at(ga.lam + (size_t)i * Ns, idx);
        }
        collide_adjoint(a, g, lam, mu, Fb);
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            const int sx = CX[i] > 0 ? xm : (CX[i] < 0 ? xp : x);
            const int sy = CY[i] > 0 ? ym : (CY[i] < 0 ? yp : y);
            const int sz = CZ[i] > 0 ? zm : (CZ[i] < 0 ? zp : z);
            *at(ga.lam_prev + (size_t)i * Ns, (uint32_t)(sx + nx * (sy + ny * sz))) = mu[i];
        }
    } else if (in) {
        const int xp = x + 1 == nx ? 0 : x + 1, xm = x == 0 ? nx - 1 : x - 1;
        const int yp = y + 1 == ny ? 0 : y + 1, ym = y == 0 ? ny - 1 : y - 1;
        const int zp = z + 1 == nz ? 0 : z + 1, zm = z == 0 ? nz - 1 : z - 1;
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            const int sx = CX[i] > 0 ? xm : (CX[i] < 0 ? xp : x);
            const int sy = CY[i] > 0 ? ym : (CY[i] < 0 ? yp : y);
            const int sz = CZ[i] > 0 ? zm : (CZ[i] < 0 ? zp : z);
            *at(ga.lam_prev + (size_t)i * Ns, (uint32_t)(sx + nx * (sy + ny * sz))) = 0.0f;
        }
    }
    // body-force part: per-tile sums in a fixed order
    __shared__ double s_red[kBlock / 64][3];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int p = 0; p < 3; ++p) Fb[p] += __shfl_xor(Fb[p], off);
    if ((tid & 63) == 0)
#pragma unroll
        for (int p = 0; p < 3; ++p) s_red[tid >> 6][p] = Fb[p];
    __syncthreads();
    if (tid < 3) {
        double v = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) v += s_red[w][tid];
        ga.dF_tile[3 * (size_t)t + tid] += v;
    }
}

__global__ __launch_bounds__(kBlock) void k_adj_reduce(const double *dF_tile, int n_tiles, double *dF)
{
    __shared__ double s_red[kBlock / 64][3];
    double v[3] = {0.0, 0.0, 0.0};
    for (int t = threadIdx.x; t < n_tiles; t += kBlock)
#pragma unroll
        for (int p = 0; p < 3; ++p) v[p] += dF_tile[3 * (size_t)t + p];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int p = 0; p < 3; ++p) v[p] += __shfl_xor(v[p], off);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int p = 0; p < 3; ++p) s_red[threadIdx.x >> 6][p] = v[p];
    __syncthreads();
    if (threadIdx.x < 3) {
        double s = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) s += s_red[w][threadIdx.x];
        dF[threadIdx.x] = s;
    }
}

}  // namespace

hipError_t launch_adj_collide(const AdjStepArgs &g, hipStream_t s)
{
    switch (g.a.tile) {
    case kTile64x2x2: hipLaunchKernelGGL((k_adj_collide<64, 2, 2>), dim3(g.a.n_tiles), dim3(kBlock), 0, s, g); break;
    case kTile32x4x2: hipLaunchKernelGGL((k_adj_collide<32, 4, 2>), dim3(g.a.n_tiles), dim3(kBlock), 0, s, g); break;
    case kTile32x2x4: hipLaunchKernelGGL((k_adj_collide<32, 2, 4>), dim3(g.a.n_tiles), dim3(kBlock), 0, s, g); break;
    case kTile16x8x2: hipLaunchKernelGGL((k_adj_collide<16, 8, 2>), dim3(g.a.n_tiles), dim3(kBlock), 0, s, g); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_adj_reduce(const double *dF_tile, int n_tiles, double *dF, hipStream_t s)
{
    hipLaunchKernelGGL(k_adj_reduce, dim3(1), dim3(kBlock), 0, s, dF_tile, n_tiles, dF);
    return hipGetLastError();
}

hipError_t launch_zieb_update(int storage, const ZiebArgs &z, hipStream_t s)
{
    const int grid = std::min(kZiebMaxBlocks, std::max(1, (z.nx * z.ny + kBlock - 1) / kBlock));
    switch (storage) {
    case 0: hipLaunchKernelGGL(k_zieb_update<0>, dim3(grid), dim3(kBlock), 0, s, z); break;
    case 1: hipLaunchKernelGGL(k_zieb_update<1>, dim3(grid), dim3(kBlock), 0, s, z); break;
    case 2: hipLaunchKernelGGL(k_zieb_update<2>, dim3(grid), dim3(kBlock), 0, s, z); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_step(int storage, const StepArgs &a, hipStream_t s)
{
    switch (storage) {
    case 0: return launch_step_s<0>(a, s);
    case 1: return launch_step_s<1>(a, s);
    case 2: return launch_step_s<2>(a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace lbm
