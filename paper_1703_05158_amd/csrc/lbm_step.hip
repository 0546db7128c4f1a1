// One D3Q19 step on gfx950: the fused step kernel and the force gather.
//
// k_step computes, for every fluid node of a 256-node tile, in one pass over
// HBM:
//  1. boundary links (near-boundary nodes only): for each link from x to a
//     solid node x + c_K (bits of the node's solid-link mask), the Bouzidi
//     value of the population I = opposite(K) that x receives (Sec. 2.3: the
//     q < 1/2 and q >= 1/2 branches and eq. moving_boundary_velocity) into
//     the thread's LDS column, and the momentum exchanged on the link
//     (Sec. 2.3 force and torque), reduced per wavefront and body into the
//     tile's LDS table;
//  2. pull streaming (the streaming equation of Sec. 2.2; the links above
//     replace their pulled values), moments (eqs. dens, momentum, with the
//     Guo half-force velocity shift), the Smagorinsky relaxation time of
//     Sec. 2.2, BGK collision with the Guo source (eq. Collision_step), store.
// The two phases never hold their working sets at the same time, which keeps
// the kernel's register budget that of the plain pull-collide.
// k_forces then forms the per-body force/torque from the per-tile sums.
//
// Forces: link contributions are summed per lane and accumulated per tile in
// LDS with FP64 LDS atomics (a small hash table for spheres, dedicated slots
// for walls).  A tile writes its sphere sums as compact
// records and its wall sums densely; k_forces sums, for each sphere, the
// records of the tiles its bounding box touches, and reduces the wall
// partials.  No global atomics on the common path.
#include "lbm_device.h"
#include "lbm_internal.h"

#include <hip/hip_runtime.h>
#include <math.h>

namespace lbm {
namespace {

using namespace dev;

struct Tables {
    int *id;              // [kRec]
    double (*v)[6];       // [kRec][6]
    double (*w)[6];       // [kMaxWalls][6]
};

// Add one body's partial sums to the tile's LDS table.
__device__ __forceinline__ void table_add(const Tables &tb, int slot, int nb, const double *v, double *overflow)
{
    if (slot >= nb) {
        double *p = tb.w[slot - nb];
#pragma unroll
        for (int c = 0; c < 6; ++c) atomicAdd(p + c, v[c]);
        return;
    }
    int j = slot & (kRec - 1);
#pragma unroll 1
    for (int probe = 0; probe < kRec; ++probe) {
        const int cur = atomicCAS(tb.id + j, -1, slot);
        if (cur == -1 || cur == slot) {
#pragma unroll
            for (int c = 0; c < 6; ++c) atomicAdd(&tb.v[j][c], v[c]);
            return;
        }
        j = (j + 1) & (kRec - 1);
    }
#pragma unroll
    for (int c = 0; c < 6; ++c) atomicAdd(overflow + 6 * slot + c, v[c]);
}

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous range of tiles so that the y/z neighbour rows a tile pulls were
// brought into the same XCD's L2 by the tiles just before it.
__device__ __forceinline__ int xcd_remap(int b, int nblocks)
{
    const int per = nblocks >> 3;
    if (b >= (per << 3)) return b;
    return (b & 7) * per + (b >> 3);
}

// One cut link, from fluid node (x, y, z) towards the solid node x + c_K
// (K = opposite(I)): the Bouzidi value of the population I that x receives,
// into LDS repl[I * kBlock] of the node's column, and the momentum handed to
// the body into acc.  `solid` is the node's solid-link mask.
template <int S>
__device__ __forceinline__ void bounce_link(const StepArgs &a, const typename Store<S>::T *src, uint32_t idx,
                                            int x, int y, int z, int I, uint32_t solid, float *repl, int &acc_id,
                                            double (&acc)[6], const Tables &tb, bool &ins)
{
    using St = Store<S>;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const size_t Ns = (size_t)a.Ns;
    const int K = opp(I);
    const int ckx = -dcx(I), cky = -dcy(I), ckz = -dcz(I);
    const uint32_t sidx = (uint32_t)(wrap_add(x, ckx, nx) + nx * (wrap_add(y, cky, ny) + ny * wrap_add(z, ckz, nz)));
    const int ob = *at(a.own, sidx);
    // own-node populations and the raw value pulled along K, issued together
    const float fk = St::ld(at(src + (size_t)K * Ns, idx));
    const float fi = St::ld(at(src + (size_t)I * Ns, idx));
    const bool back_fluid = !((solid >> K) & 1u);
    float gk = 0.f;
    if (back_fluid) {
        const uint32_t bidx =
            (uint32_t)(wrap_add(x, -ckx, nx) + nx * (wrap_add(y, -cky, ny) + ny * wrap_add(z, -ckz, nz)));
        gk = St::ld(at(src + (size_t)K * Ns, bidx));
    }
    double q, ar0, ar1, ar2, u0, u1, u2;
    if (ob < a.n_walls) {
        const double *wl = a.walls + ob * kWallStride;
        q = 0.5;
        u0 = wl[0];
        u1 = wl[1];
        u2 = wl[2];
        ar0 = (double)x + 0.5 * ckx - wl[3];
        ar1 = (double)y + 0.5 * cky - wl[4];
        ar2 = (double)z + 0.5 * ckz - wl[5];
    } else {
        const double *B = a.bodies + (ob - a.n_walls) * kBodyStride;
        const double d0 = min_image((double)x - B[0], nx);
        const double d1 = min_image((double)y - B[1], ny);
        const double d2 = min_image((double)z - B[2], nz);
        if (a.halfway) {
            q = 0.5;
        } else {
            // smallest root in (0,1] of |d + q c_K|^2 = R^2, cancellation-free form
            const double bb = d0 * ckx + d1 * cky + d2 * ckz;
            const double aa = (double)(ckx * ckx + cky * cky + ckz * ckz);
            const double cc = __dadd_rn(__dadd_rn(__dmul_rn(d0, d0), __dmul_rn(d1, d1)), __dmul_rn(d2, d2)) -
                              __dmul_rn(B[9], B[9]);
            const double disc = fmax(bb * bb - aa * cc, 0.0);
            q = fmin(fmax(cc / (sqrt(disc) - bb), 0.0), 1.0);
        }
        ar0 = d0 + q * ckx;
        ar1 = d1 + q * cky;
        ar2 = d2 + q * ckz;
        u0 = B[3] + (B[7] * ar2 - B[8] * ar1);
        u1 = B[4] + (B[8] * ar0 - B[6] * ar2);
        u2 = B[5] + (B[6] * ar1 - B[7] * ar0);
    }
    // moving-boundary term along the reflected direction I = -K
    const float wk = (float)wgt(K);
    const float mw = wk * a.rho0 * (float)(-(ckx * u0 + cky * u1 + ckz * u2));
    const float qf = (float)q;
    float val;
    if (q < 0.5) {
        val = back_fluid ? 2.0f * qf * fk + (1.0f - 2.0f * qf) * gk + 6.0f * mw : fk + 6.0f * mw;
    } else {
        const float h = 0.5f / qf;
        val = h * fk + (1.0f - h) * fi + (3.0f / qf) * mw;
    }
    repl[I * kBlock] = val;
    // momentum handed to the body along c_K (full populations)
    const double mom = (double)fk + (double)val + 2.0 * (double)wk * (double)a.rho0;
    const double F0 = mom * ckx, F1 = mom * cky, F2 = mom * ckz;
    const int slot = ob < a.n_walls ? a.nb + ob : ob - a.n_walls;
    if (slot != acc_id) {
        if (acc_id >= 0) {
            table_add(tb, acc_id, a.nb, acc, a.overflow);
            ins = true;
        }
        acc_id = slot;
#pragma unroll
        for (int j = 0; j < 6; ++j) acc[j] = 0.0;
    }
    acc[0] += F0;
    acc[1] += F1;
    acc[2] += F2;
    acc[3] += ar1 * F2 - ar2 * F1;
    acc[4] += ar2 * F0 - ar0 * F2;
    acc[5] += ar0 * F1 - ar1 * F0;
}

// 5 waves per SIMD: the register budget of the boundary-link phase without spills
template <int S, int TX, int TY, int TZ>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(5, 5))) void k_step(StepArgs a)
{
    static_assert(TX * TY * TZ == kBlock, "tile must hold one workgroup");
    using St = Store<S>;
    using T = typename St::T;
    const T *__restrict__ src = static_cast<const T *>(a.src);
    T *__restrict__ dst = static_cast<T *>(a.dst);
    const size_t Ns = (size_t)a.Ns;
    const int nx = a.nx, ny = a.ny, nz = a.nz;

    __shared__ int s_id[kRec];
    __shared__ double s_v[kRec][6];
    __shared__ double s_w[kMaxWalls][6];
    __shared__ float s_g[kQ * kBlock];  // boundary-link values, one column per thread
    __shared__ uint32_t s_mask[kBlock]; // solid-link mask per thread's node
    __shared__ int s_off[kBlock + 1];   // exclusive prefix sum of link counts
    const Tables tb{s_id, s_v, s_w};

    const int tid = threadIdx.x;
    for (int j = tid; j < kRec; j += kBlock) s_id[j] = -1;
    for (int j = tid; j < kRec * 6; j += kBlock) (&s_v[0][0])[j] = 0.0;
    for (int j = tid; j < kMaxWalls * 6; j += kBlock) (&s_w[0][0])[j] = 0.0;
    if (blockIdx.x == 0)
        for (int j = tid; j < a.n_walls * 6; j += kBlock) a.out[a.nb * 6 + j] = 0.0;
    __syncthreads();

    const int t = xcd_remap(blockIdx.x, gridDim.x);
    const int r = t / a.ntx;
    const int x = (t - r * a.ntx) * TX + tid % TX;
    const int y = (r % a.nty) * TY + (tid / TX) % TY;
    const int z = (r / a.nty) * TZ + tid / (TX * TY);
    const bool in = x < nx && y < ny && z < nz;
    const uint32_t idx = in ? (uint32_t)(x + nx * (y + ny * z)) : 0u;
    // owner code and link mask together (the mask is meaningful for kNear only)
    const uint16_t o = in ? *at(a.own, idx) : uint16_t(0);
    const uint32_t nm = in ? *at(a.nmask, idx) : 0u;
    const bool fluid = o >= kNear;
    const uint32_t solid = o == kNear ? nm : 0u;

    // pull: population i arrives from x - c_i; in flight during the link phase
    float g[kQ];
    if (fluid) {
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
    }

    // 1. boundary links, spread over the workgroup: link j belongs to the
    //    node of thread p with s_off[p] <= j < s_off[p + 1]
    int acc_id = -1;
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    bool ins = false;
    {
        const int cnt = __popc(solid);
        // inclusive scan within the wavefront, then across the 4 wavefronts
        const int lane = __lane_id(), wv = tid >> 6;
        int incl = cnt;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const int v = __shfl_up(incl, off);
            if (lane >= off) incl += v;
        }
        s_mask[tid] = solid;
        if (lane == 63) s_off[kBlock - 4 + wv] = incl;  // wavefront totals, parked at the end
        __syncthreads();
        int base = 0;
        for (int w = 0; w < wv; ++w) base += s_off[kBlock - 4 + w];
        const int total = s_off[kBlock - 4] + s_off[kBlock - 3] + s_off[kBlock - 2] + s_off[kBlock - 1];
        __syncthreads();
        s_off[tid] = base + incl - cnt;
        if (tid == 0) s_off[kBlock] = total;
        __syncthreads();
        const int r0 = t / a.ntx;
        const int bx = (t - r0 * a.ntx) * TX, by = (r0 % a.nty) * TY, bz = (r0 / a.nty) * TZ;
#pragma unroll 1
        for (int j = tid; j < total; j += kBlock) {
            int lo = 0, hi = kBlock;  // largest p with s_off[p] <= j
            while (hi - lo > 1) {
                const int mid = (lo + hi) >> 1;
                if (s_off[mid] <= j) lo = mid;
                else hi = mid;
            }
            const int p = lo;
            uint32_t msk = s_mask[p];
            for (int k = j - s_off[p]; k > 0; --k) msk &= msk - 1;
            const int I = __builtin_ctz(msk);
            const int px = bx + p % TX, py = by + (p / TX) % TY, pz = bz + p / (TX * TY);
            bounce_link<S>(a, src, (uint32_t)(px + nx * (py + ny * pz)), px, py, pz, I, s_mask[p], s_g + p, acc_id,
                           acc, tb, ins);
        }
    }
    // each lane's partial sums straight into the tile's LDS table
    if (acc_id >= 0) {
        table_add(tb, acc_id, a.nb, acc, a.overflow);
        ins = true;
    }
    __syncthreads();  // link values of every node of the tile are in LDS

    // 2. collide, store
    if (fluid) {
        if (solid) {
#pragma unroll
            for (int i = 1; i < kQ; ++i)
                if ((solid >> i) & 1u) g[i] = s_g[i * kBlock + tid];
        }

        // moments in opposite pairs (i, i+9): even and odd parts
        float pe[10], po[10];
#pragma unroll
        for (int i = 1; i <= 9; ++i) {
            pe[i] = g[i] + g[i + 9];
            po[i] = g[i] - g[i + 9];
        }
        float rd = g[0], jx = 0.f, jy = 0.f, jz = 0.f;
        float sxx = 0.f, syy = 0.f, szz = 0.f, sxy = 0.f, sxz = 0.f, syz = 0.f;
#pragma unroll
        for (int i = 1; i <= 9; ++i) {
            rd += pe[i];
            if (CX[i]) jx += CX[i] * po[i];
            if (CY[i]) jy += CY[i] * po[i];
            if (CZ[i]) jz += CZ[i] * po[i];
            if (CX[i]) sxx += pe[i];
            if (CY[i]) syy += pe[i];
            if (CZ[i]) szz += pe[i];
            if (CX[i] * CY[i]) sxy += CX[i] * CY[i] * pe[i];
            if (CX[i] * CZ[i]) sxz += CX[i] * CZ[i] * pe[i];
            if (CY[i] * CZ[i]) syz += CY[i] * CZ[i] * pe[i];
        }
        const float rho = a.rho0 + rd;
        const float ir = __builtin_amdgcn_rcpf(rho);
        const float ux = (jx + 0.5f * a.fx) * ir;
        const float uy = (jy + 0.5f * a.fy) * ir;
        const float uz = (jz + 0.5f * a.fz) * ir;
        // second moment of f - feq
        const float third = 1.0f / 3.0f;
        const float pxx = sxx - rd * third - rho * ux * ux;
        const float pyy = syy - rd * third - rho * uy * uy;
        const float pzz = szz - rd * third - rho * uz * uz;
        const float pxy = sxy - rho * ux * uy;
        const float pxz = sxz - rho * ux * uz;
        const float pyz = syz - rho * uy * uz;
        const float Qn = pxx * pxx + pyy * pyy + pzz * pzz + 2.0f * (pxy * pxy + pxz * pxz + pyz * pyz);
        const float tau = 0.5f * (a.tau0 + __builtin_sqrtf(a.tau0 * a.tau0 + a.smag_k * __builtin_sqrtf(Qn) * ir));
        const float om = __builtin_amdgcn_rcpf(tau);
        const float om1 = 1.0f - om;
        const float cf = 1.0f - 0.5f * om;
        const float uu = ux * ux + uy * uy + uz * uz;
        const float uF = ux * a.fx + uy * a.fy + uz * a.fz;
        if (a.flag && !(rho > 0.f && isfinite(uu))) atomicOr(a.flag, 1);
        {   // rest population: equilibrium deviation w0 (rd - 1.5 rho uu), source -3 w0 cf uF
            const float w = (float)wgt(0);
            St::st(at(dst, idx), om1 * g[0] + om * w * (rd - 1.5f * rho * uu) - 3.0f * w * cf * uF);
        }
#pragma unroll
        for (int i = 1; i <= 9; ++i) {
            const float w = (float)wgt(i);
            const float cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
            const float cF = CX[i] * a.fx + CY[i] * a.fy + CZ[i] * a.fz;
            // equilibrium deviation: even w (rd + rho (4.5 cu^2 - 1.5 uu)), odd 3 w rho cu
            // Guo source: even w cf (9 cu cF - 3 uF), odd 3 w cf cF
            const float ev = om * w * (rd + rho * (4.5f * cu * cu - 1.5f * uu)) + w * cf * (9.0f * cu * cF - 3.0f * uF);
            const float od = 3.0f * w * (om * rho * cu + cf * cF);
            St::st(at(dst + (size_t)i * Ns, idx), om1 * g[i] + ev + od);
            St::st(at(dst + (size_t)(i + 9) * Ns, idx), om1 * g[i + 9] + ev - od);
        }
    }

    // tile records: compact sphere sums, dense wall sums
    const int nw6 = a.n_walls * 6;
    if (__syncthreads_or(ins)) {
        if (tid < 64) {
            const int id = tid < kRec ? s_id[tid] : -1;
            const unsigned long long msk = __ballot(id >= 0);
            if (id >= 0) {
                const int p = t * kRec + __popcll(msk & ((1ull << tid) - 1ull));
                a.rec_id[p] = id;
#pragma unroll
                for (int c = 0; c < 6; ++c) a.rec_v[6 * p + c] = s_v[tid][c];
            }
            if (tid == 0) a.rec_n[t] = (int)__popcll(msk);
            for (int j = tid; j < nw6; j += 64) a.wallpart[(size_t)t * nw6 + j] = s_w[j / 6][j % 6];
        }
    } else {
        if (tid == 0) a.rec_n[t] = 0;
        for (int j = tid; j < nw6; j += kBlock) a.wallpart[(size_t)t * nw6 + j] = 0.0;
    }
}

// Tiles along one axis that hold nodes within one link of [c - r, c + r]:
// `cnt` consecutive tile indices (mod ntile) starting at `s`.
__device__ __forceinline__ void axis_tiles(double c, double r, int n, int T, int ntile, int &s, int &cnt)
{
    const int lo = (int)floor(c - r) - 1, hi = (int)ceil(c + r) + 1;
    if (hi - lo + 1 > n - T) {
        s = 0;
        cnt = ntile;
        return;
    }
    s = wrap1(lo, n) / T;
    const int e = wrap1(hi, n) / T;
    cnt = e >= s ? e - s + 1 : e + ntile - s + 1;
}

constexpr int kWallGroups = 64;

__global__ __launch_bounds__(64) void k_forces(StepArgs a, int TX, int TY, int TZ)
{
    const int b = blockIdx.x, lane = threadIdx.x;
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (b < a.nb) {
        const double *B = a.bodies + b * kBodyStride;
        if (body_ok(B, a.nx, a.ny, a.nz)) {
            int sx, cx, sy, cy, sz, cz;
            axis_tiles(B[0], B[9], a.nx, TX, a.ntx, sx, cx);
            axis_tiles(B[1], B[9], a.ny, TY, a.nty, sy, cy);
            axis_tiles(B[2], B[9], a.nz, TZ, a.ntz, sz, cz);
            const int total = cx * cy * cz;
            for (int c = lane; c < total; c += 64) {
                const int i = c % cx, j = (c / cx) % cy, k = c / (cx * cy);
                const int tx = (sx + i) % a.ntx, ty = (sy + j) % a.nty, tz = (sz + k) % a.ntz;
                const int tt = tx + a.ntx * (ty + a.nty * tz);
                const int n = a.rec_n[tt];
                for (int rr = 0; rr < n; ++rr) {
                    const int p = tt * kRec + rr;
                    if (a.rec_id[p] == b)
#pragma unroll
                        for (int q = 0; q < 6; ++q) v[q] += a.rec_v[6 * p + q];
                }
            }
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
#pragma unroll
            for (int q = 0; q < 6; ++q) v[q] += __shfl_xor(v[q], off);
        if (lane < 6) {
            const double o = a.overflow[6 * b + lane];
            a.out[6 * b + lane] = v[lane] + o;
            a.overflow[6 * b + lane] = 0.0;
        }
        return;
    }
    const int w = (b - a.nb) / kWallGroups, gi = (b - a.nb) % kWallGroups;
    const int nw6 = a.n_walls * 6;
    for (int t = gi * 64 + lane; t < a.n_tiles; t += kWallGroups * 64)
#pragma unroll
        for (int q = 0; q < 6; ++q) v[q] += a.wallpart[(size_t)t * nw6 + 6 * w + q];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1)
#pragma unroll
        for (int q = 0; q < 6; ++q) v[q] += __shfl_xor(v[q], off);
    if (lane < 6) atomicAdd(a.out + 6 * (a.nb + w) + lane, v[lane]);
}

template <int S>
hipError_t launch_step_s(const StepArgs &a, hipStream_t s)
{
    if (a.tile == kTile64x2x2)
        hipLaunchKernelGGL((k_step<S, 64, 2, 2>), dim3(a.n_tiles), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL((k_step<S, 32, 4, 2>), dim3(a.n_tiles), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_step(int storage, const StepArgs &a, hipStream_t s)
{
    switch (storage) {
    case 0: return launch_step_s<0>(a, s);
    case 1: return launch_step_s<1>(a, s);
    case 2: return launch_step_s<2>(a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_forces(const StepArgs &a, hipStream_t s)
{
    const int grid = a.nb + a.n_walls * kWallGroups;
    if (grid <= 0) return hipSuccess;
    const int TX = a.tile == kTile64x2x2 ? 64 : 32, TY = a.tile == kTile64x2x2 ? 2 : 4, TZ = 2;
    hipLaunchKernelGGL(k_forces, dim3(grid), dim3(64), 0, s, a, TX, TY, TZ);
    return hipGetLastError();
}

}  // namespace lbm
