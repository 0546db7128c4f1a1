// Arithmetic of one cut lattice link (Sec. 2.3), shared by the boundary-link
// pass and the fused step kernel so that both give the same values bit for
// bit.  Contraction into fused multiply-adds is off here: the two kernels
// would otherwise be free to fuse different products.
//
// Notation: x is the fluid node, I the population it receives, K =
// opposite(I) the direction from x to the solid node p = x + c_K = x - c_I.
// Sphere links take q, the fraction of the link x -> p inside the fluid, and
// the wall velocity at x_b = x + q c_K; walls close their links at q = 1/2.
#pragma once

#include "lbm_device.h"

namespace lbm {
namespace dev {

// Kinematics of a solid as its links see it, from a record of kBodyStride
// doubles {X[3], V[3], Omega[3], R}: a sphere's centre, velocity, angular
// velocity and radius, or a wall's torque reference point and velocity
// (Omega = 0, R unused).  Reference point in FP64, the rest in FP32.
struct SphereK {
    double X0, X1, X2;
    float V0, V1, V2, W0, W1, W2, R2;
};

__device__ __forceinline__ SphereK sphere_k(const double *B)
{
    SphereK k;
    k.X0 = B[0];
    k.X1 = B[1];
    k.X2 = B[2];
    k.V0 = (float)B[3];
    k.V1 = (float)B[4];
    k.V2 = (float)B[5];
    k.W0 = (float)B[6];
    k.W1 = (float)B[7];
    k.W2 = (float)B[8];
    k.R2 = (float)(B[9] * B[9]);
    return k;
}

// Geometry of the link (x, I) of a solid: the offset d = x - X (the minimum
// image for a sphere; plain for a wall, whose arm is taken about its
// reference point), the link fraction q and the moving-boundary term
// mw = w_K rho0 (c_I . u_w) with u_w = V + Omega x (x_b - X).  q is the
// exact sphere fraction when exact_q, else 1/2 (walls, halfway mode).
struct LinkGeo {
    double d0, d1, d2;
    float q, mw;
};

__device__ __forceinline__ LinkGeo link_geo(const SphereK &k, bool exact_q, bool sphere, float rho0, int x, int y,
                                            int z, int nx, int ny, int nz, int I)
{
#pragma clang fp contract(off)
    const int cx = dcx(I), cy = dcy(I), cz = dcz(I);  // c_I = -c_K
    LinkGeo l;
    l.d0 = (double)x - k.X0;
    l.d1 = (double)y - k.X1;
    l.d2 = (double)z - k.X2;
    if (sphere) {
        l.d0 = min_image(l.d0, nx);
        l.d1 = min_image(l.d1, ny);
        l.d2 = min_image(l.d2, nz);
    }
    // the offset rounded once from FP64; q and the wall velocity in FP32
    const float e0 = (float)l.d0, e1 = (float)l.d1, e2 = (float)l.d2;
    if (exact_q) {
        // smallest root in (0, 1] of |d + q c_K|^2 = R^2, cancellation-free form
        const float bb = -(e0 * cx + e1 * cy + e2 * cz);
        const float aa = (float)(cx * cx + cy * cy + cz * cz);
        const float cc = (e0 * e0 + e1 * e1 + e2 * e2) - k.R2;
        const float disc = fmaxf(bb * bb - aa * cc, 0.0f);
        // (the hardware square root and reciprocal, each within 1 ulp)
        l.q = fminf(fmaxf(cc * __builtin_amdgcn_rcpf(__builtin_amdgcn_sqrtf(disc) - bb), 0.0f), 1.0f);
    } else {
        l.q = 0.5f;
    }
    // wall point x_b = x + q c_K relative to X, and its velocity
    const float f0 = e0 - l.q * cx, f1 = e1 - l.q * cy, f2 = e2 - l.q * cz;
    const float u0 = k.V0 + (k.W1 * f2 - k.W2 * f1);
    const float u1 = k.V1 + (k.W2 * f0 - k.W0 * f2);
    const float u2 = k.V2 + (k.W0 * f1 - k.W1 * f0);
    l.mw = (float)wgt(opp(I)) * rho0 * (cx * u0 + cy * u1 + cz * u2);
    return l;
}

// The population x receives along I across the link (the two branches of
// Sec. 2.3 with the moving-boundary term): fk = P(x)[K], fa = P(x)[I],
// fb = P(x + c_I)[K] when the node behind x is fluid (behind), else unused.
// At q = 1/2 both branches give fk + 6 mw (bounce-back at the link
// midpoint), which is taken exactly, without fa.
__device__ __forceinline__ float link_value(float q, float fk, float fa, float fb, bool behind, float mw)
{
#pragma clang fp contract(off)
    if (q < 0.5f) return behind ? 2.0f * q * fk + (1.0f - 2.0f * q) * fb + 6.0f * mw : fk + 6.0f * mw;
    if (q == 0.5f) return fk + 6.0f * mw;
    const float rq = __builtin_amdgcn_rcpf(q);
    const float h = 0.5f * rq;
    return h * fk + (1.0f - h) * fa + (3.0f * rq) * mw;
}

// Momentum handed to the body across the link, as full populations:
// P(x)[K] + f_I(x) + 2 w rho0 (the two stored deviations plus their
// weights), in FP64.
__device__ __forceinline__ double link_momentum(float fk, float vr, int I, float rho0)
{
#pragma clang fp contract(off)
    return (double)fk + (double)vr + 2.0 * wgt(I) * (double)rho0;
}

// Force mom c_K on the body and its torque about the lever arm
// x_b - X = d - q c_I, as t[6] = {F, T} (FP64).  The force is parallel to
// c_I, so (d - q c_I) x F = d x F: the arm is taken as d.
__device__ __forceinline__ void link_force_terms(double mom, int I, const LinkGeo &l, double (&t)[6])
{
#pragma clang fp contract(off)
    const int cx = dcx(I), cy = dcy(I), cz = dcz(I);
    const double a0 = l.d0, a1 = l.d1, a2 = l.d2;
    const double F0 = -mom * cx, F1 = -mom * cy, F2 = -mom * cz;
    t[0] = F0;
    t[1] = F1;
    t[2] = F2;
    t[3] = a1 * F2 - a2 * F1;
    t[4] = a2 * F0 - a0 * F2;
    t[5] = a0 * F1 - a1 * F0;
}

// The same terms added to acc[6].
__device__ __forceinline__ void link_force(double mom, int I, const LinkGeo &l, double (&acc)[6])
{
#pragma clang fp contract(off)
    double t[6];
    link_force_terms(mom, I, l, t);
#pragma unroll
    for (int c = 0; c < 6; ++c) acc[c] += t[c];
}

// Exclusive prefix of `cnt` (0 <= cnt < 64) over the workgroup and the total
// (wtot: one int per wavefront in LDS).  Contains a barrier.
__device__ __forceinline__ int block_scan(int cnt, int *wtot, int &tot)
{
    constexpr int kWaves = kBlock / 64;
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    // the wavefront's prefix bit plane by bit plane (cnt < 64): the lanes
    // below this one with bit b set, from a ballot
    int pos = 0, wsum = 0;
#pragma unroll
    for (int b = 0; b < 6; ++b) {
        const unsigned long long m = __ballot((cnt >> b) & 1);
        pos += (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u)) << b;
        wsum += __popcll(m) << b;
    }
    if (lane == 0) wtot[wv] = wsum;
    __syncthreads();
    tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        const int t = wtot[w];
        if (w < wv) pos += t;
        tot += t;
    }
    return pos;
}

}  // namespace dev
}  // namespace lbm
