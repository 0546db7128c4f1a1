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
//    owner map (loads issued together with the population loads, two links
//    per thread in flight) and reduces force and torque itself;
//  - wall links do not change while the walls stay: their fluid nodes are
//    listed once per (wall, direction); workgroups take chunks of the list
//    and write per-chunk sums that the step kernel adds up per wall.
#include "lbm_device.h"
#include "lbm_internal.h"
#include "lbm_linkmath.h"

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

// Candidate link (p, I) from the fluid node x = p + c_I to the node p of a
// sphere.  The geometry comes first (it needs no memory): q decides which
// second population the interpolation uses, so a link loads the owner codes
// of p, x (and of the node behind x when q < 1/2) and two populations, all in
// one round trip.  Populations read at a node that turns out to be solid are
// discarded (the load may see a link value being written there).
struct LinkLoad {
    int I;
    uint32_t pi;
    uint16_t op, ox, ob;
    float fk, f2;         // f2: P(x)[I] when q >= 1/2, else P(x - c_K)[K]
    LinkGeo g;            // offset from the centre, q, moving-boundary term
};

template <int S>
__device__ __forceinline__ LinkLoad link_load(const LinkArgs &a, const typename Store<S>::T *pop,
                                              const SphereK &k, int px, int py, int pz, int I)
{
    using St = Store<S>;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const size_t Ns = (size_t)a.Ns;
    const int cx = dcx(I), cy = dcy(I), cz = dcz(I);  // c_I = -c_K
    const int K = opp(I);
    LinkLoad l;
    l.I = I;
    const int x = wrap1(px + cx, nx), y = wrap1(py + cy, ny), z = wrap1(pz + cz, nz);
    l.pi = (uint32_t)(px + nx * (py + ny * pz));
    const uint32_t xi = (uint32_t)(x + nx * (y + ny * z));
    l.g = link_geo(k, !a.halfway, true, a.rho0, x, y, z, nx, ny, nz, I);
    l.op = *at(a.own, l.pi);
    l.ox = *at(a.own, xi);
    l.fk = St::ld(at(pop + (size_t)K * Ns, xi));
    if (l.g.q < 0.5f) {
        const uint32_t bi = (uint32_t)(wrap1(x + cx, nx) + nx * (wrap1(y + cy, ny) + ny * wrap1(z + cz, nz)));
        l.ob = *at(a.own, bi);
        l.f2 = St::ld(at(pop + (size_t)K * Ns, bi));
    } else {
        l.ob = kFluid;
        l.f2 = St::ld(at(pop + (size_t)I * Ns, xi));
    }
    return l;
}

// The link, if it is one (p owned by the sphere `own_b`, x fluid): the
// Bouzidi value into slot I of p and the momentum into acc (lever arm and
// sums in FP64).
template <int S>
__device__ __forceinline__ void link_finish(const LinkArgs &a, typename Store<S>::T *pop, uint16_t own_b,
                                            const LinkLoad &l, double (&acc)[6])
{
    using St = Store<S>;
    if (l.op != own_b || l.ox < kVacated) return;
    const int I = l.I;
    const bool behind = l.ob >= kVacated;
    const float vr = St::round(link_value(l.g.q, l.fk, l.f2, l.f2, behind, l.g.mw));
    St::st(at(pop + (size_t)I * (size_t)a.Ns, l.pi), vr);
    link_force(link_momentum(l.fk, vr, I, a.rho0), I, l.g, acc);
}

constexpr int kItemCap = 4096;   // candidate links held at once
constexpr int kRoundNodes = 224; // box nodes per round when a sphere has more (224 * 18 <= kItemCap)

// Per-direction link counts packed two to a word: word w holds the opposite
// directions w + 1 (bits 0-15) and w + 10 (bits 16-31); word kCW is the
// total.
constexpr int kCW = (kQ - 1) / 2;

constexpr int kMaskCap = 4096;  // box nodes whose candidate masks are kept between the two passes

struct SphereLds {
    uint32_t item[kItemCap];  // box node index << 5 | I
    uint32_t mask[kMaskCap];  // candidate directions of each box node
    int wtot[kWaves];
    uint32_t ctot[kWaves][kCW + 1];
};

// Candidate links of box node k: p is within a margin of the ball and more
// than R - 1.5 deep at most (deeper nodes have no neighbour outside), and
// (p, I) when p + c_I lies outside the ball by the same margin.  The margin
// covers the FP32 rounding, so every link is a candidate; the owner map then
// decides exactly.
__device__ __forceinline__ uint32_t cand_mask(const SphereK &k, float mg, float in2, float dx, float dy, float dz)
{
    const float d2 = dx * dx + dy * dy + dz * dz;
    uint32_t lm = 0;
    if (d2 <= k.R2 + mg && d2 >= in2) {
        // |d + c|^2 > R^2 - mg  <=>  2 d.c > R^2 - mg - d^2 - |c|^2
        const float t = k.R2 - mg - d2;
        const float ax = 2.0f * dx, ay = 2.0f * dy, az = 2.0f * dz;
#pragma unroll
        for (int i = 1; i < kQ; ++i) {
            const float dc = CX[i] * ax + CY[i] * ay + CZ[i] * az;
            const float cc = (float)(CX[i] * CX[i] + CY[i] * CY[i] + CZ[i] * CZ[i]);
            if (dc > t - cc) lm |= 1u << i;
        }
    }
    return lm;
}

// The same for box node kk (x fastest), with its coordinates.
__device__ __forceinline__ uint32_t candidates(const LinkArgs &a, const Box &bx, const SphereK &k, float mg,
                                               float in2, int kk, int &px, int &py, int &pz)
{
    const int kx = kk % bx.ex, kr = kk / bx.ex;
    px = wrap1(bx.x0 + kx, a.nx);
    py = wrap1(bx.y0 + kr % bx.ey, a.ny);
    pz = wrap1(bx.z0 + kr / bx.ey, a.nz);
    const float dx = (float)min_image((double)px - k.X0, a.nx);
    const float dy = (float)min_image((double)py - k.X1, a.ny);
    const float dz = (float)min_image((double)pz - k.X2, a.nz);
    return cand_mask(k, mg, in2, dx, dy, dz);
}

// Offset of box coordinate v (unwrapped) from the centre coordinate c.  A
// box spans at most 2R + 1 < n - 1 nodes around the centre, so this is the
// minimum image.
__device__ __forceinline__ float box_off(int v, double c) { return (float)((double)v - c); }

// Number of bits that hold 0 .. e - 1.
__device__ __forceinline__ int field_bits(int e) { return e > 1 ? 32 - __clz(e - 1) : 1; }

// Exclusive prefix over the workgroup of each of the NW words (in v) and
// their totals (in tot).
template <int NW>
__device__ __forceinline__ void block_scan_words(uint32_t (&v)[NW], uint32_t (*wtot)[NW], uint32_t (&tot)[NW])
{
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    uint32_t incl[NW];
#pragma unroll
    for (int w = 0; w < NW; ++w) incl[w] = v[w];
#pragma unroll
    for (int off = 1; off < 64; off <<= 1)
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            const uint32_t t = __shfl_up(incl[w], off);
            if (lane >= off) incl[w] += t;
        }
    if (lane == 63)
#pragma unroll
        for (int w = 0; w < NW; ++w) wtot[wv][w] = incl[w];
    __syncthreads();
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        uint32_t pos = incl[w] - v[w], t = 0;
#pragma unroll
        for (int q = 0; q < kWaves; ++q) {
            const uint32_t u = wtot[q][w];
            if (q < wv) pos += u;
            t += u;
        }
        v[w] = pos;
        tot[w] = t;
    }
}

// Box node of a list item (node << 5 | I): packed coordinates kx | ky << wx
// | kz << (wx + wy) when wx > 0, else the box index.
__device__ __forceinline__ void item_node(const LinkArgs &a, const Box &bx, int wx, int wy, uint32_t it, int &px,
                                          int &py, int &pz)
{
    const uint32_t v = it >> 5;
    int kx, ky, kz;
    if (wx > 0) {
        kx = (int)(v & ((1u << wx) - 1u));
        ky = (int)((v >> wx) & ((1u << wy) - 1u));
        kz = (int)(v >> (wx + wy));
    } else {
        kx = (int)v % bx.ex;
        ky = ((int)v / bx.ex) % bx.ey;
        kz = (int)v / (bx.ex * bx.ey);
    }
    px = wrap1(bx.x0 + kx, a.nx);
    py = wrap1(bx.y0 + ky, a.ny);
    pz = wrap1(bx.z0 + kz, a.nz);
}

// Links of the candidates listed in item[0, tot), two per thread at a time.
template <int S>
__device__ __forceinline__ void process_items(const LinkArgs &a, typename Store<S>::T *pop, const Box &bx,
                                              const SphereK &k, uint16_t own_b, const uint32_t *item, int tot,
                                              int wx, int wy, double (&acc)[6])
{
#pragma unroll 1
    for (int j = threadIdx.x; j < tot; j += 2 * kBlock) {
        const int j2 = j + kBlock;
        int px, py, pz;
        const uint32_t ia = item[j];
        item_node(a, bx, wx, wy, ia, px, py, pz);
        const LinkLoad la = link_load<S>(a, pop, k, px, py, pz, (int)(ia & 31));
        LinkLoad lb;
        lb.op = 0;  // no second link: fails the ownership test
        if (j2 < tot) {
            const uint32_t ib = item[j2];
            item_node(a, bx, wx, wy, ib, px, py, pz);
            lb = link_load<S>(a, pop, k, px, py, pz, (int)(ib & 31));
        }
        link_finish<S>(a, pop, own_b, la, acc);
        if (j2 < tot) link_finish<S>(a, pop, own_b, lb, acc);
    }
}

// Sphere b.  Candidates of the whole box are listed at once when they fit
// in kItemCap, else in rounds of kRoundNodes box nodes.
template <int S>
__device__ __forceinline__ void sphere_block(const LinkArgs &a, int b, SphereLds &L, double (*s_red)[6])
{
    using St = Store<S>;
    typename St::T *pop = static_cast<typename St::T *>(a.pop);
    const double *B = a.bodies + (size_t)b * kBodyStride;
    const int tid = threadIdx.x;
    double acc[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (body_ok(B, a.nx, a.ny, a.nz)) {
        const Box bx = body_box(B, 0);
        const int total = bx.ex * bx.ey * bx.ez;
        const uint16_t own_b = (uint16_t)(a.n_walls + b);
        const SphereK k = sphere_k(B);
        const float mg = 0.01f + 1e-5f * k.R2;
        const float ri = (float)B[9] - 1.5f;
        const float in2 = ri > 0.0f ? ri * ri - mg : -1.0f;
        int px, py, pz, tot;
        // Each thread takes a contiguous run of box nodes.  The list is
        // ordered by direction, then by box node, so that the lanes of one
        // load instruction read neighbouring nodes of one population array;
        // each direction I is followed by its opposite, since the links of
        // both read the arrays I and opposite(I).
        const int per = (total + kBlock - 1) / kBlock;
        const int k0 = tid * per, k1 = min(total, k0 + per);
        uint32_t cw[kCW + 1];
#pragma unroll
        for (int w = 0; w <= kCW; ++w) cw[w] = 0;
        const bool keep = total <= kMaskCap;
        // box coordinates of node k0, then stepped along the run
        int kx = k0 % bx.ex, ky = (k0 / bx.ex) % bx.ey, kz = k0 / (bx.ex * bx.ey);
        float dy = box_off(bx.y0 + ky, k.X1), dz = box_off(bx.z0 + kz, k.X2);
        for (int kk = k0; kk < k1; ++kk) {
            const uint32_t lm = cand_mask(k, mg, in2, box_off(bx.x0 + kx, k.X0), dy, dz);
            if (++kx == bx.ex) {
                kx = 0;
                if (++ky == bx.ey) {
                    ky = 0;
                    dz = box_off(bx.z0 + ++kz, k.X2);
                }
                dy = box_off(bx.y0 + ky, k.X1);
            }
            if (keep) L.mask[kk] = lm;
#pragma unroll
            for (int w = 0; w < kCW; ++w) cw[w] += ((lm >> (w + 1)) & 1u) | (((lm >> (w + 10)) & 1u) << 16);
            cw[kCW] += __popc(lm);
        }
        uint32_t ct[kCW + 1];
        block_scan_words<kCW + 1>(cw, L.ctot, ct);
        tot = (int)ct[kCW];
        if (tot <= kItemCap) {
            // no field exceeds kItemCap, so none carried into its neighbour
            uint32_t pos[kQ - 1];
            uint32_t base = 0;
#pragma unroll
            for (int w = 0; w < kCW; ++w) {
                pos[w] = base + (cw[w] & 0xFFFFu);
                base += ct[w] & 0xFFFFu;
                pos[w + 9] = base + (cw[w] >> 16);
                base += ct[w] >> 16;
            }
            // list items carry the packed box coordinates when they fit
            const int wx = field_bits(bx.ex), wy = field_bits(bx.ey);
            const bool packed = wx + wy + field_bits(bx.ez) <= 27;
            kx = k0 % bx.ex;
            ky = (k0 / bx.ex) % bx.ey;
            kz = k0 / (bx.ex * bx.ey);
            dy = box_off(bx.y0 + ky, k.X1);
            dz = box_off(bx.z0 + kz, k.X2);
            for (int kk = k0; kk < k1; ++kk) {
                const uint32_t lm = keep ? L.mask[kk] : cand_mask(k, mg, in2, box_off(bx.x0 + kx, k.X0), dy, dz);
                const uint32_t node =
                    packed ? (uint32_t)kx | ((uint32_t)ky << wx) | ((uint32_t)kz << (wx + wy)) : (uint32_t)kk;
#pragma unroll
                for (int I = 1; I < kQ; ++I)
                    if ((lm >> I) & 1u) L.item[pos[I - 1]++] = (node << 5) | (uint32_t)I;
                if (++kx == bx.ex) {
                    kx = 0;
                    if (++ky == bx.ey) {
                        ky = 0;
                        dz = box_off(bx.z0 + ++kz, k.X2);
                    }
                    dy = box_off(bx.y0 + ky, k.X1);
                }
            }
            __syncthreads();
            process_items<S>(a, pop, bx, k, own_b, L.item, tot, packed ? wx : 0, wy, acc);
        } else {
            for (int base = 0; base < total; base += kRoundNodes) {
                __syncthreads();  // item and wtot of the previous pass are free
                const int kk = base + tid;
                uint32_t lm = 0;
                if (tid < kRoundNodes && kk < total) lm = candidates(a, bx, k, mg, in2, kk, px, py, pz);
                int pos = block_scan(__popc(lm), L.wtot, tot);
                while (lm) {
                    const int I = __builtin_ctz(lm);
                    lm &= lm - 1;
                    L.item[pos++] = ((uint32_t)kk << 5) | (uint32_t)I;
                }
                __syncthreads();
                process_items<S>(a, pop, bx, k, own_b, L.item, tot, 0, 0, acc);
            }
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
    const SphereK wk = sphere_k(a.wrec + (size_t)w * kBodyStride);
    // force and torque sums; the chunk's kWallChunk / kBlock links per
    // thread have their loads in flight together
    constexpr int U = kWallChunk / kBlock;
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
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
        const LinkGeo g = link_geo(wk, false, false, a.rho0, (int)x, (int)y, (int)z, nx, ny, a.nz, I);
        const float vr = St::round(link_value(g.q, fk[u], fk[u], fk[u], false, g.mw));
        St::st(at(pop + (size_t)I * Ns, (uint32_t)(sx + nx * (sy + ny * sz))), vr);
        link_force(link_momentum(fk[u], vr, I, a.rho0), I, g, v);
    }
    block_sum<6>(v, s_red);
    if (threadIdx.x == 0) {
        double *o = a.wl_part + 6 * (size_t)blk;
#pragma unroll
        for (int c = 0; c < 6; ++c) o[c] = v[c];
    }
}

template <int S>
__global__ __launch_bounds__(kBlock) void k_links(LinkArgs a)
{
    __shared__ SphereLds L;
    __shared__ double s_red[kWaves][6];
    const int b = blockIdx.x;
    if (b < a.nb) {
        // workgroups go round-robin over the 8 XCDs: each XCD takes runs
        // of consecutive spheres in processing order (Morton order of the
        // centres when the host set them), so that neighbouring spheres,
        // which share population lines, share an L2
        const int sb = xcd_remap(b, a.nb);
        sphere_block<S>(a, a.order ? a.order[sb] : sb, L, s_red);
    }
    else
        wall_block<S>(a, b - a.nb, s_red);
}

// ---- reverse mode of the link pass ---------------------------------------
//
// Transpose of the boundary links for the gradient of the summed sphere
// drag, with the spheres fixed and the same candidate enumeration and FP32
// q as the forward pass.  A link (p, I) of sphere b from the fluid node
// x = p + c_I wrote f_I(x) = a_k P(x)[K] + a_b P(x - c_K)[K] + a_i P(x)[I]
// + a_w w_K rho0 c_I . u_w(V_b), with (a_k, a_b, a_i, a_w) = (2q, 1 - 2q, 0, 6)
// for q < 1/2 with a fluid node behind x, (1, 0, 0, 6) without, and
// (1/(2q), 0, 1 - 1/(2q), 3/q) for q >= 1/2.  Given the adjoint
// m of f_I(x) (mu), the link adds a_k m, a_b m and a_i m to the adjoints of
// those three populations and a_w w_K rho0 c_I m to dJ/dV_b.  Without mu the
// weight is that of the objective itself, J = sum_b F_b,x with F_b = sum
// (P(x)[K] + f_I(x)) c_K: m = c_K,x, plus c_K,x on P(x)[K] directly.
// Several links can reach one population (thin gaps), so the adds are atomic.
__device__ __forceinline__ void adj_sphere_block(const AdjLinkArgs &g, int b, SphereLds &L, double (*s_red)[6])
{
    const LinkArgs &a = g.a;
    const double *B = a.bodies + (size_t)b * kBodyStride;
    const int nx = a.nx, ny = a.ny, nz = a.nz;
    const size_t Ns = (size_t)a.Ns;
    const int tid = threadIdx.x;
    double acc[3] = {0.0, 0.0, 0.0};
    if (body_ok(B, nx, ny, nz)) {
        const Box bx = body_box(B, 0);
        const int total = bx.ex * bx.ey * bx.ez;
        const uint16_t own_b = (uint16_t)(a.n_walls + b);
        const SphereK k = sphere_k(B);
        const float mg = 0.01f + 1e-5f * k.R2;
        const float ri = (float)B[9] - 1.5f;
        const float in2 = ri > 0.0f ? ri * ri - mg : -1.0f;
        for (int base = 0; base < total; base += kRoundNodes) {
            __syncthreads();
            const int kk = base + tid;
            int px = 0, py = 0, pz = 0, tot;
            uint32_t lm = 0;
            if (tid < kRoundNodes && kk < total) lm = candidates(a, bx, k, mg, in2, kk, px, py, pz);
            int pos = block_scan(__popc(lm), L.wtot, tot);
            while (lm) {
                const int I = __builtin_ctz(lm);
                lm &= lm - 1;
                L.item[pos++] = ((uint32_t)kk << 5) | (uint32_t)I;
            }
            __syncthreads();
            for (int j = tid; j < tot; j += kBlock) {
                const uint32_t it = L.item[j];
                const int kj = (int)(it >> 5), I = (int)(it & 31), K = opp(I);
                px = wrap1(bx.x0 + kj % bx.ex, nx);
                py = wrap1(bx.y0 + (kj / bx.ex) % bx.ey, ny);
                pz = wrap1(bx.z0 + kj / (bx.ex * bx.ey), nz);
                const int cx = dcx(I), cy = dcy(I), cz = dcz(I);
                const int x = wrap1(px + cx, nx), y = wrap1(py + cy, ny), z = wrap1(pz + cz, nz);
                const uint32_t pi = (uint32_t)(px + nx * (py + ny * pz));
                const uint32_t xi = (uint32_t)(x + nx * (y + ny * z));
                if (*at(a.own, pi) != own_b || *at(a.own, xi) < kVacated) continue;
                const float q = link_geo(k, !a.halfway, true, a.rho0, x, y, z, nx, ny, nz, I).q;
                const float ckx = (float)(-cx);
                const float m = g.mu ? *at(g.mu + (size_t)I * Ns, pi) : ckx;
                float ak, ab = 0.f, ai = 0.f, aw;
                uint32_t bi = 0;
                if (q < 0.5f) {
                    bi = (uint32_t)(wrap1(x + cx, nx) + nx * (wrap1(y + cy, ny) + ny * wrap1(z + cz, nz)));
                    if (*at(a.own, bi) >= kVacated) {
                        ak = 2.0f * q;
                        ab = 1.0f - 2.0f * q;
                    } else {
                        ak = 1.0f;
                    }
                    aw = 6.0f;
                } else {
                    const float h = 0.5f / q;
                    ak = h;
                    ai = 1.0f - h;
                    aw = 3.0f / q;
                }
                atomicAdd(at(g.lam + (size_t)K * Ns, xi), ak * m + (g.mu ? 0.0f : ckx));
                if (ab != 0.0f) atomicAdd(at(g.lam + (size_t)K * Ns, bi), ab * m);
                if (ai != 0.0f) atomicAdd(at(g.lam + (size_t)I * Ns, xi), ai * m);
                const double wv = (double)(aw * (float)wgt(K) * a.rho0 * m);
                acc[0] += wv * cx;
                acc[1] += wv * cy;
                acc[2] += wv * cz;
            }
        }
    }
    block_sum<3>(acc, s_red);
    if (tid == 0)
#pragma unroll
        for (int c = 0; c < 3; ++c) g.dV[3 * (size_t)b + c] += acc[c];
}

__global__ __launch_bounds__(kBlock) void k_adj_links(AdjLinkArgs g)
{
    __shared__ SphereLds L;
    __shared__ double s_red[kWaves][6];
    adj_sphere_block(g, blockIdx.x, L, s_red);
}

}  // namespace

hipError_t launch_adj_links(const AdjLinkArgs &g, hipStream_t s)
{
    if (g.a.nb <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_adj_links, dim3(g.a.nb), dim3(kBlock), 0, s, g);
    return hipGetLastError();
}

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

}  // namespace lbm
