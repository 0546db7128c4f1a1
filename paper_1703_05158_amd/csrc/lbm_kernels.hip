// gfx950 kernels of the D3Q19 moving-boundary lattice Boltzmann step.
//
// The hot kernel k_step performs, for every fluid node and in one pass over
// HBM: pull streaming (Sec. 2.2, streaming equation), interpolated
// bounce-back with the moving-boundary term on links cut by solids
// (Sec. 2.3, Bouzidi q < 1/2 and q >= 1/2 branches and eq.
// moving_boundary_velocity), moments (eqs. dens, momentum, with the Guo
// half-force velocity shift), the Smagorinsky relaxation time (Sec. 2.2),
// BGK collision with the Guo source (eq. Collision_step) and the
// momentum-exchange force/torque reduction per body (Sec. 2.3).
//
// Data layout (structure of arrays): populations pop[i][n], i = 0..18 in
// Table 1 order, n = x + nx*(y + ny*z), stored as deviations
// g_i = f_i - w_i rho0 in fp32, fp16 or bf16; owner map uint16 per node.
// One thread owns one node; a workgroup owns 256 consecutive nodes, so every
// population access of a wavefront is a contiguous 64-element run (shifted by
// +-1 element for directions with c_x != 0, absorbed by the caches).
// Solid nodes are neither read nor written: only the rasteriser refills a
// node that a sphere uncovers.
//
// The rasteriser keeps the owner map incrementally: vacate the previous
// geometry's sphere nodes, stamp the new spheres (atomic minimum, so walls and
// lower sphere indices win), refill uncovered nodes with the equilibrium at
// rho0 and the velocity they had as solids (the solid-side Maxwell
// equilibrium of Sec. 2.3), and refresh the near-boundary flags around every
// sphere that moved.
#include "lbm_internal.h"

#include <hip/hip_runtime.h>
#include <math.h>

namespace lbm {

FastDiv make_fastdiv(uint32_t d)
{
    FastDiv f;
    f.d = d;
    uint32_t l = 0;
    while ((1ull << l) < d) ++l;
    f.s = l;
    f.m = (uint32_t)((((1ull << l) - d) << 32) / d + 1);
    return f;
}

namespace {

// Table 1 of the paper.
constexpr int CX[kQ] = {0, -1, 0, 0, -1, -1, -1, -1, 0, 0, 1, 0, 0, 1, 1, 1, 1, 0, 0};
constexpr int CY[kQ] = {0, 0, -1, 0, -1, 1, 0, 0, -1, -1, 0, 1, 0, 1, -1, 0, 0, 1, 1};
constexpr int CZ[kQ] = {0, 0, 0, -1, 0, 0, -1, 1, -1, 1, 0, 0, 1, 0, 0, 1, -1, 1, -1};

constexpr uint64_t pack_dir(const int (&c)[kQ])
{
    uint64_t v = 0;
    for (int i = 0; i < kQ; ++i) v |= (uint64_t)(c[i] + 1) << (2 * i);
    return v;
}
constexpr uint64_t kPX = pack_dir(CX), kPY = pack_dir(CY), kPZ = pack_dir(CZ);

// Runtime-indexed table lookups (boundary path only) without memory traffic.
__device__ __forceinline__ int dcx(int i) { return (int)((kPX >> (2 * i)) & 3) - 1; }
__device__ __forceinline__ int dcy(int i) { return (int)((kPY >> (2 * i)) & 3) - 1; }
__device__ __forceinline__ int dcz(int i) { return (int)((kPZ >> (2 * i)) & 3) - 1; }
__device__ __forceinline__ int opp(int i) { return i == 0 ? 0 : (i <= 9 ? i + 9 : i - 9); }

// Weights: w0 = 1/3, axis directions (1,2,3,10,11,12) 1/18, others 1/36.
__host__ __device__ constexpr double wgt(int i)
{
    return i == 0 ? 1.0 / 3.0 : (((0x1C0Eu >> i) & 1u) ? 1.0 / 18.0 : 1.0 / 36.0);
}

// ---- storage of deviations ------------------------------------------------
template <int S> struct Store;
template <> struct Store<0> {
    using T = float;
    static __device__ __forceinline__ float ld(const T *p) { return *p; }
    static __device__ __forceinline__ void st(T *p, float v) { *p = v; }
};
template <> struct Store<1> {
    using T = _Float16;
    static __device__ __forceinline__ float ld(const T *p) { return (float)*p; }
    static __device__ __forceinline__ void st(T *p, float v) { *p = (_Float16)v; }
};
template <> struct Store<2> {  // bfloat16 held as raw bits, round-to-nearest-even
    using T = uint16_t;
    static __device__ __forceinline__ float ld(const T *p) { return __uint_as_float((uint32_t)*p << 16); }
    static __device__ __forceinline__ void st(T *p, float v)
    {
        uint32_t u = __float_as_uint(v);
        if ((u & 0x7f800000u) == 0x7f800000u)
            *p = (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
        else
            *p = (uint16_t)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
    }
};

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv &f)
{
    return (uint32_t)(((uint64_t)__umulhi(n, f.m) + n) >> f.s);
}

__device__ __forceinline__ int wrap_add(int a, int d, int n)
{
    int r = a + d;
    return r < 0 ? r + n : (r >= n ? r - n : r);
}

__device__ __forceinline__ double min_image(double d, double L)
{
    if (d > 0.5 * L) d -= L;
    else if (d < -0.5 * L) d += L;
    return d;
}

// Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous slab of nodes so that the y/z neighbours a block pulls were
// brought into the same XCD's L2 by its predecessors.
__device__ __forceinline__ int xcd_remap(int b, int nblocks)
{
    const int per = nblocks >> 3;
    if (b >= (per << 3)) return b;
    return (b & 7) * per + (b >> 3);
}

__device__ __forceinline__ void flush_acc(double *gacc, int id, const double *v)
{
    double *p = gacc + 6 * id;
#pragma unroll
    for (int j = 0; j < 6; ++j) atomicAdd(p + j, v[j]);
}

// ---- the fused step -------------------------------------------------------
template <int S>
__global__ __launch_bounds__(kBlock) void k_step(StepArgs a)
{
    using St = Store<S>;
    using T = typename St::T;
    const T *__restrict__ src = static_cast<const T *>(a.src);
    T *__restrict__ dst = static_cast<T *>(a.dst);
    const uint16_t *__restrict__ own = a.own;
    const size_t N = (size_t)a.N;

    __shared__ float sg[kQ][kBlock];  // per-thread populations on the boundary path

    const int tid = threadIdx.x;
    const int idx = xcd_remap(blockIdx.x, a.nblocks) * kBlock + tid;
    const bool in = idx < a.N;
    const uint16_t o = in ? own[idx] : uint16_t(0);

    int acc_id = -1;
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};

    if (in && o >= kNear) {
        const int nx = a.nx, ny = a.ny, nz = a.nz;
        const uint32_t t = fdiv((uint32_t)idx, a.div_nx);
        const int x = idx - (int)t * nx;
        const int z = (int)fdiv(t, a.div_ny);
        const int y = (int)t - z * ny;
        const int xp = x + 1 == nx ? 0 : x + 1, xm = x == 0 ? nx - 1 : x - 1;
        const int yp = y + 1 == ny ? 0 : y + 1, ym = y == 0 ? ny - 1 : y - 1;
        const int zp = z + 1 == nz ? 0 : z + 1, zm = z == 0 ? nz - 1 : z - 1;

        // pull: population i arrives from x - c_i
        float g[kQ];
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            const int sx = CX[i] > 0 ? xm : (CX[i] < 0 ? xp : x);
            const int sy = CY[i] > 0 ? ym : (CY[i] < 0 ? yp : y);
            const int sz = CZ[i] > 0 ? zm : (CZ[i] < 0 ? zp : z);
            g[i] = St::ld(src + (size_t)i * N + (sx + nx * (sy + ny * sz)));
        }

        if (o == kNear) {
            // Links to solid nodes: replace the pulled value of population
            // i = opposite(k) by the Bouzidi interpolation (Sec. 2.3).
            uint32_t solid = 0;
#pragma unroll
            for (int i = 1; i < kQ; ++i) {
                const int sx = CX[i] > 0 ? xm : (CX[i] < 0 ? xp : x);
                const int sy = CY[i] > 0 ? ym : (CY[i] < 0 ? yp : y);
                const int sz = CZ[i] > 0 ? zm : (CZ[i] < 0 ? zp : z);
                if (own[sx + nx * (sy + ny * sz)] < kVacated) solid |= 1u << i;
            }
#pragma unroll
            for (int i = 0; i < kQ; ++i) sg[i][tid] = g[i];
            const float rho0 = a.rho0;
            uint32_t m = solid;
            while (m) {
                const int i = __builtin_ctz(m);
                m &= m - 1;
                const int k = opp(i);
                const int ckx = -dcx(i), cky = -dcy(i), ckz = -dcz(i);
                const int sidx = wrap_add(x, ckx, nx) + nx * (wrap_add(y, cky, ny) + ny * wrap_add(z, ckz, nz));
                const int ob = own[sidx];
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
                        // smallest root in (0,1] of |d + q c_k|^2 = R^2
                        const double bb = d0 * ckx + d1 * cky + d2 * ckz;
                        const double aa = (double)(ckx * ckx + cky * cky + ckz * ckz);
                        const double cc = __dadd_rn(__dadd_rn(__dmul_rn(d0, d0), __dmul_rn(d1, d1)),
                                                    __dmul_rn(d2, d2)) - __dmul_rn(B[9], B[9]);
                        const double disc = fmax(bb * bb - aa * cc, 0.0);
                        q = cc / (sqrt(disc) - bb);
                        q = fmin(fmax(q, 0.0), 1.0);
                    }
                    ar0 = d0 + q * ckx;
                    ar1 = d1 + q * cky;
                    ar2 = d2 + q * ckz;
                    u0 = B[3] + (B[7] * ar2 - B[8] * ar1);
                    u1 = B[4] + (B[8] * ar0 - B[6] * ar2);
                    u2 = B[5] + (B[6] * ar1 - B[7] * ar0);
                }
                // moving-boundary term along the reflected direction i = -k
                const float ciu = (float)(-(ckx * u0 + cky * u1 + ckz * u2));
                const float wk = (float)wgt(k);
                const float mw = wk * rho0 * ciu;
                const float fk = St::ld(src + (size_t)k * N + idx);
                const float qf = (float)q;
                float val;
                if (q < 0.5) {
                    if (!((solid >> k) & 1u))
                        val = 2.0f * qf * fk + (1.0f - 2.0f * qf) * sg[k][tid] + 6.0f * mw;
                    else
                        val = fk + 6.0f * mw;
                } else {
                    const float fi = St::ld(src + (size_t)i * N + idx);
                    const float h = 0.5f / qf;
                    val = h * fk + (1.0f - h) * fi + (3.0f / qf) * mw;
                }
                sg[i][tid] = val;
                // momentum handed to the body along c_k (full populations)
                const double mom = (double)fk + (double)val + 2.0 * wgt(k) * (double)rho0;
                const double F0 = mom * ckx, F1 = mom * cky, F2 = mom * ckz;
                const int slot = ob < a.n_walls ? a.nb + ob : ob - a.n_walls;
                if (slot != acc_id) {
                    if (acc_id >= 0) flush_acc(a.acc, acc_id, acc);
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
#pragma unroll
            for (int i = 0; i < kQ; ++i) g[i] = sg[i][tid];
        }

        // moments of the deviations
        float rd = 0.f, jx = 0.f, jy = 0.f, jz = 0.f;
        float sxx = 0.f, syy = 0.f, szz = 0.f, sxy = 0.f, sxz = 0.f, syz = 0.f;
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            rd += g[i];
            if (CX[i]) jx += CX[i] * g[i];
            if (CY[i]) jy += CY[i] * g[i];
            if (CZ[i]) jz += CZ[i] * g[i];
            if (CX[i]) sxx += g[i];
            if (CY[i]) syy += g[i];
            if (CZ[i]) szz += g[i];
            if (CX[i] * CY[i]) sxy += CX[i] * CY[i] * g[i];
            if (CX[i] * CZ[i]) sxz += CX[i] * CZ[i] * g[i];
            if (CY[i] * CZ[i]) syz += CY[i] * CZ[i] * g[i];
        }
        const float rho = a.rho0 + rd;
        const float ir = 1.0f / rho;
        const float ux = (jx + 0.5f * a.fx) * ir;
        const float uy = (jy + 0.5f * a.fy) * ir;
        const float uz = (jz + 0.5f * a.fz) * ir;
        // non-equilibrium second moment: sum c c (f - feq)
        const float third = 1.0f / 3.0f;
        const float pxx = sxx - rd * third - rho * ux * ux;
        const float pyy = syy - rd * third - rho * uy * uy;
        const float pzz = szz - rd * third - rho * uz * uz;
        const float pxy = sxy - rho * ux * uy;
        const float pxz = sxz - rho * ux * uz;
        const float pyz = syz - rho * uy * uz;
        const float Qn = pxx * pxx + pyy * pyy + pzz * pzz + 2.0f * (pxy * pxy + pxz * pxz + pyz * pyz);
        const float tau = 0.5f * (a.tau0 + sqrtf(a.tau0 * a.tau0 + a.smag_k * sqrtf(Qn) * ir));
        const float om = 1.0f / tau;
        const float cf = 1.0f - 0.5f * om;
        const float uu = ux * ux + uy * uy + uz * uz;
        const float uF = ux * a.fx + uy * a.fy + uz * a.fz;
        if (a.flag && !(rho > 0.f && isfinite(uu))) atomicOr(a.flag, 1);
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            const float w = (float)wgt(i);
            const float cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
            const float cF = CX[i] * a.fx + CY[i] * a.fy + CZ[i] * a.fz;
            const float geq = w * (rd + rho * (3.0f * cu + 4.5f * cu * cu - 1.5f * uu));
            const float sgu = w * cf * (3.0f * (cF - uF) + 9.0f * cu * cF);
            St::st(dst + (size_t)i * N + idx, g[i] - om * (g[i] - geq) + sgu);
        }
    }

    // Force/torque: one atomic per body per wavefront (grouped by owner id).
    unsigned long long pending = __ballot(acc_id >= 0);
    const int lane = __lane_id();
    while (pending) {
        const int leader = __ffsll((long long)pending) - 1;
        const int id = __shfl(acc_id, leader);
        const bool mine = acc_id == id;
        double v[6];
#pragma unroll
        for (int j = 0; j < 6; ++j) v[j] = mine ? acc[j] : 0.0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1)
#pragma unroll
            for (int j = 0; j < 6; ++j) v[j] += __shfl_xor(v[j], off);
        if (lane == leader) flush_acc(a.acc, id, v);
        if (mine) acc_id = -1;
        pending = __ballot(acc_id >= 0);
    }
}

// ---- geometry -------------------------------------------------------------
__device__ __forceinline__ bool body_ok(const double *B, int nx, int ny, int nz)
{
    const double lim = 0.5 * (double)min(nx, min(ny, nz)) - 1.0;
    return B[9] > 0.0 && B[9] < lim && B[0] >= 0.0 && B[0] < nx && B[1] >= 0.0 && B[1] < ny &&
           B[2] >= 0.0 && B[2] < nz;
}

// |p - X|^2 <= R^2 with the minimum image, as a plain product-sum
// evaluated left to right without fused multiply-add.
__device__ __forceinline__ bool inside(const double *B, int px, int py, int pz, int nx, int ny, int nz)
{
    const double dx = min_image((double)px - B[0], nx);
    const double dy = min_image((double)py - B[1], ny);
    const double dz = min_image((double)pz - B[2], nz);
    const double d2 = __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
    return d2 <= __dmul_rn(B[9], B[9]);
}

struct Box {
    int x0, y0, z0, ex, ey, ez;
};

__device__ __forceinline__ Box body_box(const double *B, int pad)
{
    Box b;
    b.x0 = (int)ceil(B[0] - B[9]) - pad;
    b.y0 = (int)ceil(B[1] - B[9]) - pad;
    b.z0 = (int)ceil(B[2] - B[9]) - pad;
    b.ex = (int)floor(B[0] + B[9]) + pad - b.x0 + 1;
    b.ey = (int)floor(B[1] + B[9]) + pad - b.y0 + 1;
    b.ez = (int)floor(B[2] + B[9]) + pad - b.z0 + 1;
    return b;
}

__device__ __forceinline__ int wrapc(int a, int n) { return ((a % n) + n) % n; }

__device__ __forceinline__ void atomic_min_u16(uint16_t *addr, uint16_t val)
{
    unsigned int *w = (unsigned int *)((uintptr_t)addr & ~(uintptr_t)3);
    const unsigned int sh = ((uintptr_t)addr & 2) ? 16u : 0u;
    unsigned int old = __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while (true) {
        const unsigned int cur = (old >> sh) & 0xffffu;
        if (cur <= val) return;
        const unsigned int nw = (old & ~(0xffffu << sh)) | ((unsigned int)val << sh);
        const unsigned int prev = atomicCAS(w, old, nw);
        if (prev == old) return;
        old = prev;
    }
}

__global__ __launch_bounds__(kBlock) void k_walls_init(const uint8_t *wall, uint16_t *own, int N)
{
    const int n = blockIdx.x * kBlock + threadIdx.x;
    if (n < N) own[n] = wall[n] ? (uint16_t)(wall[n] - 1) : kFluid;
}

__device__ __forceinline__ uint16_t fluid_flag(const uint16_t *own, int x, int y, int z, int nx, int ny, int nz)
{
#pragma unroll
    for (int i = 1; i < kQ; ++i) {
        const int s = wrap_add(x, CX[i], nx) + nx * (wrap_add(y, CY[i], ny) + ny * wrap_add(z, CZ[i], nz));
        if (own[s] < kVacated) return kNear;
    }
    return kFluid;
}

__global__ __launch_bounds__(kBlock) void k_flags_full(GeomArgs g)
{
    const int n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= g.N) return;
    const uint16_t o = g.own[n];
    if (o < kNear) return;
    const int x = n % g.nx, y = (n / g.nx) % g.ny, z = n / (g.nx * g.ny);
    const uint16_t f = fluid_flag(g.own, x, y, z, g.nx, g.ny, g.nz);
    if (f != o) g.own[n] = f;
}

__global__ __launch_bounds__(kBlock) void k_vacate(GeomArgs g)
{
    const int b = blockIdx.x;
    const double *B = g.bodies + b * kBodyStride;
    if (!body_ok(B, g.nx, g.ny, g.nz)) return;
    const uint16_t id = (uint16_t)(g.n_walls + b);
    const Box bx = body_box(B, 0);
    const int total = bx.ex * bx.ey * bx.ez;
    for (int t = threadIdx.x; t < total; t += kBlock) {
        const int px = wrapc(bx.x0 + t % bx.ex, g.nx);
        const int py = wrapc(bx.y0 + (t / bx.ex) % bx.ey, g.ny);
        const int pz = wrapc(bx.z0 + t / (bx.ex * bx.ey), g.nz);
        const int n = px + g.nx * (py + g.ny * pz);
        if (g.own[n] == id) g.own[n] = (uint16_t)(kVacated | id);
    }
}

__global__ __launch_bounds__(kBlock) void k_stamp(GeomArgs g)
{
    const int b = blockIdx.x;
    const double *B = g.bodies + b * kBodyStride;
    if (!body_ok(B, g.nx, g.ny, g.nz)) return;
    const uint16_t id = (uint16_t)(g.n_walls + b);
    const Box bx = body_box(B, 0);
    const int total = bx.ex * bx.ey * bx.ez;
    for (int t = threadIdx.x; t < total; t += kBlock) {
        const int px = wrapc(bx.x0 + t % bx.ex, g.nx);
        const int py = wrapc(bx.y0 + (t / bx.ex) % bx.ey, g.ny);
        const int pz = wrapc(bx.z0 + t / (bx.ex * bx.ey), g.nz);
        if (inside(B, px, py, pz, g.nx, g.ny, g.nz)) atomic_min_u16(g.own + (px + g.nx * (py + g.ny * pz)), id);
    }
}

// Deviation of the equilibrium at rho0 and velocity u: w_i rho0 (3 c.u + 4.5 (c.u)^2 - 1.5 u.u).
__device__ __forceinline__ double eq_dev(int i, double rho0, double u0, double u1, double u2)
{
    const double cu = dcx(i) * u0 + dcy(i) * u1 + dcz(i) * u2;
    return wgt(i) * rho0 * (3.0 * cu + 4.5 * cu * cu - 1.5 * (u0 * u0 + u1 * u1 + u2 * u2));
}

__device__ __forceinline__ void sphere_velocity(const double *B, int px, int py, int pz, int nx, int ny, int nz,
                                                double &u0, double &u1, double &u2)
{
    const double r0 = min_image((double)px - B[0], nx);
    const double r1 = min_image((double)py - B[1], ny);
    const double r2 = min_image((double)pz - B[2], nz);
    u0 = B[3] + (B[7] * r2 - B[8] * r1);
    u1 = B[4] + (B[8] * r0 - B[6] * r2);
    u2 = B[5] + (B[6] * r1 - B[7] * r0);
}

template <int S>
__global__ __launch_bounds__(kBlock) void k_refill(GeomArgs g)
{
    using St = Store<S>;
    typename St::T *pop = static_cast<typename St::T *>(g.pop);
    const int b = blockIdx.x;
    const double *B = g.bodies + b * kBodyStride;
    if (!body_ok(B, g.nx, g.ny, g.nz)) return;
    const uint16_t tag = (uint16_t)(kVacated | (g.n_walls + b));
    const Box bx = body_box(B, 0);
    const int total = bx.ex * bx.ey * bx.ez;
    for (int t = threadIdx.x; t < total; t += kBlock) {
        const int px = wrapc(bx.x0 + t % bx.ex, g.nx);
        const int py = wrapc(bx.y0 + (t / bx.ex) % bx.ey, g.ny);
        const int pz = wrapc(bx.z0 + t / (bx.ex * bx.ey), g.nz);
        const int n = px + g.nx * (py + g.ny * pz);
        if (g.own[n] != tag) continue;
        double u0, u1, u2;
        sphere_velocity(B, px, py, pz, g.nx, g.ny, g.nz, u0, u1, u2);
        for (int i = 0; i < kQ; ++i) St::st(pop + (size_t)i * g.N + n, (float)eq_dev(i, g.rho0, u0, u1, u2));
        g.own[n] = kFluid;
    }
}

__global__ __launch_bounds__(kBlock) void k_flags_bodies(GeomArgs g)
{
    const int j = blockIdx.x;
    const double *B = j < g.nb ? g.bodies + j * kBodyStride : g.bodies2 + (j - g.nb) * kBodyStride;
    if (!body_ok(B, g.nx, g.ny, g.nz)) return;
    const Box bx = body_box(B, 1);
    const int total = bx.ex * bx.ey * bx.ez;
    for (int t = threadIdx.x; t < total; t += kBlock) {
        const int px = wrapc(bx.x0 + t % bx.ex, g.nx);
        const int py = wrapc(bx.y0 + (t / bx.ex) % bx.ey, g.ny);
        const int pz = wrapc(bx.z0 + t / (bx.ex * bx.ey), g.nz);
        const int n = px + g.nx * (py + g.ny * pz);
        const uint16_t o = g.own[n];
        if (o < kNear) continue;
        const uint16_t f = fluid_flag(g.own, px, py, pz, g.nx, g.ny, g.nz);
        if (f != o) g.own[n] = f;
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
    if (g.own[n] < kNear) {
        for (int i = 0; i < kQ; ++i) St::st(pop + i * N + n, 0.0f);
        return;
    }
    const double r = rho ? rho[n] : (double)g.rho0;
    const double u0 = u ? u[n] : 0.0, u1 = u ? u[N + n] : 0.0, u2 = u ? u[2 * N + n] : 0.0;
    const double uu = u0 * u0 + u1 * u1 + u2 * u2;
    for (int i = 0; i < kQ; ++i) {
        const double cu = dcx(i) * u0 + dcy(i) * u1 + dcz(i) * u2;
        const double dev = wgt(i) * (r - (double)g.rho0) + wgt(i) * r * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu);
        St::st(pop + i * N + n, (float)dev);
    }
}

__device__ __forceinline__ void solid_velocity(const GeomArgs &g, const double *walls, uint16_t o, int px,
                                               int py, int pz, double &u0, double &u1, double &u2)
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
    if (o >= kNear) {
        out[n] = (double)St::ld(pop + (size_t)dir * g.N + n) + wgt(dir) * (double)g.rho0;
        return;
    }
    const int px = n % g.nx, py = (n / g.nx) % g.ny, pz = n / (g.nx * g.ny);
    double u0, u1, u2;
    solid_velocity(g, walls, o, px, py, pz, u0, u1, u2);
    out[n] = wgt(dir) * (double)g.rho0 + eq_dev(dir, g.rho0, u0, u1, u2);
}

template <int S>
__global__ __launch_bounds__(kBlock) void k_import_pop(int N, int dir, float rho0, const double *in, void *popv)
{
    using St = Store<S>;
    typename St::T *pop = static_cast<typename St::T *>(popv);
    const int n = blockIdx.x * kBlock + threadIdx.x;
    if (n < N) St::st(pop + (size_t)dir * N + n, (float)(in[n] - wgt(dir) * (double)rho0));
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
    if (o >= kNear) {
        double r = 0.0, j0 = 0.0, j1 = 0.0, j2 = 0.0;
        for (int i = 0; i < kQ; ++i) {
            const double f = (double)St::ld(pop + i * N + n) + wgt(i) * (double)g.rho0;
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
    if (n < N) out[n] = own[n] >= kNear ? -1 : (int32_t)own[n];
}

__global__ __launch_bounds__(kBlock) void k_zero(double *p, int n)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) p[i] = 0.0;
}

__global__ __launch_bounds__(kBlock) void k_count_fluid(const uint16_t *own, int N, unsigned long long *count)
{
    const int n = blockIdx.x * kBlock + threadIdx.x;
    const unsigned long long mask = __ballot(n < N && own[n] >= kNear);
    if (__lane_id() == 0 && mask) atomicAdd(count, (unsigned long long)__popcll(mask));
}

inline int nblk(long n) { return (int)((n + kBlock - 1) / kBlock); }

template <template <int> class K, typename... A>
hipError_t dispatch(int storage, dim3 grid, hipStream_t s, A... args)
{
    switch (storage) {
    case 0: hipLaunchKernelGGL(K<0>::fn, grid, dim3(kBlock), 0, s, args...); break;
    case 1: hipLaunchKernelGGL(K<1>::fn, grid, dim3(kBlock), 0, s, args...); break;
    case 2: hipLaunchKernelGGL(K<2>::fn, grid, dim3(kBlock), 0, s, args...); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

template <int S> struct StepK { static constexpr auto fn = k_step<S>; };
template <int S> struct RefillK { static constexpr auto fn = k_refill<S>; };
template <int S> struct InitK { static constexpr auto fn = k_init_pop<S>; };
template <int S> struct ExportK { static constexpr auto fn = k_export_pop<S>; };
template <int S> struct ImportK { static constexpr auto fn = k_import_pop<S>; };
template <int S> struct MacroK { static constexpr auto fn = k_export_macro<S>; };

}  // namespace

hipError_t launch_step(int storage, const StepArgs &a, hipStream_t s)
{
    if (a.nblocks <= 0) return hipSuccess;
    return dispatch<StepK>(storage, dim3(a.nblocks), s, a);
}

hipError_t launch_walls_init(const uint8_t *wall, uint16_t *own, int N, hipStream_t s)
{
    hipLaunchKernelGGL(k_walls_init, dim3(nblk(N)), dim3(kBlock), 0, s, wall, own, N);
    return hipGetLastError();
}

hipError_t launch_flags_full(const GeomArgs &g, hipStream_t s)
{
    hipLaunchKernelGGL(k_flags_full, dim3(nblk(g.N)), dim3(kBlock), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_vacate(const GeomArgs &g, hipStream_t s)
{
    if (g.nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_vacate, dim3(g.nb), dim3(kBlock), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_stamp(const GeomArgs &g, hipStream_t s)
{
    if (g.nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_stamp, dim3(g.nb), dim3(kBlock), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_refill(int storage, const GeomArgs &g, hipStream_t s)
{
    if (g.nb <= 0) return hipSuccess;
    return dispatch<RefillK>(storage, dim3(g.nb), s, g);
}

hipError_t launch_flags_bodies(const GeomArgs &g, hipStream_t s)
{
    if (g.nb + g.nb2 <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_flags_bodies, dim3(g.nb + g.nb2), dim3(kBlock), 0, s, g);
    return hipGetLastError();
}

hipError_t launch_init_pop(int storage, const GeomArgs &g, const double *rho, const double *u, hipStream_t s)
{
    return dispatch<InitK>(storage, dim3(nblk(g.N)), s, g, rho, u);
}

hipError_t launch_export_pop(int storage, const GeomArgs &g, const double *walls, int dir, double *out,
                             hipStream_t s)
{
    return dispatch<ExportK>(storage, dim3(nblk(g.N)), s, g, walls, dir, out);
}

hipError_t launch_import_pop(int storage, int N, int dir, float rho0, const double *in, void *pop, hipStream_t s)
{
    return dispatch<ImportK>(storage, dim3(nblk(N)), s, N, dir, rho0, in, pop);
}

hipError_t launch_export_macro(int storage, const GeomArgs &g, const double *walls, double fx, double fy,
                               double fz, double *rho, double *u, hipStream_t s)
{
    return dispatch<MacroK>(storage, dim3(nblk(g.N)), s, g, walls, fx, fy, fz, rho, u);
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
    hipLaunchKernelGGL(k_count_fluid, dim3(nblk(N)), dim3(kBlock), 0, s, own, N, count);
    return hipGetLastError();
}

}  // namespace lbm
