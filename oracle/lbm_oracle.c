/*
 * FP64 CPU oracle of one D3Q19 lattice Boltzmann step with Smagorinsky
 * relaxation, Bouzidi velocity-corrected bounce-back on moving spheres and
 * voxel walls, and momentum-exchange force/torque per body.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * HIP library is checked against.  It shares no code with the library; only
 * the test suite, the benchmark's CPU baseline and the smoke check load it.
 *
 * Everything is in lattice units (Sec. 2.2: spacing = time step = 1) and
 * double precision, evaluated in the order the paper states the method:
 *   - velocity set and weights: Table 1 and the weights given under the
 *     discrete equilibrium (Sec. 2.2);
 *   - moments: eqs. (dens), (momentum), with the half-force shift of the
 *     Guo forcing (an addition: the paper has no body-force term);
 *   - equilibrium: eq. (Equilibre_Maxwell_Boltzmann), c_s^2 = 1/3;
 *   - BGK collision: eq. (Collision_step), with tau replaced by the
 *     Smagorinsky tau* of Sec. 2.2 (Hou et al. closure);
 *   - streaming: the streaming equation of Sec. 2.2, in pull form;
 *   - boundary: Bouzidi interpolation for q < 1/2 and q >= 1/2 and the
 *     moving-boundary term eq. (moving_boundary_velocity), Sec. 2.3;
 *   - forces: momentum exchange, Sec. 2.3 (force and torque equations).
 * Readings of silent or garbled passages are those listed in the design
 * notes (sign of the moving-wall term taken along the reflected direction
 * with the reference density; force on the body from the actually reflected
 * population; solid-node populations = equilibrium at the reference density
 * and the solid velocity; tau* = (tau0 + sqrt(tau0^2 + 18 sqrt2 C^2 sqrt(Q)/rho))/2).
 *
 * Owner codes (int32 per node): -1 fluid, 0..W-1 wall object, W+b sphere b.
 * Node (x,y,z) has index x + nx*(y + ny*z); populations are [19][N].
 * Compile with -ffp-contract=off: the solid/fluid test must be the plain
 * product-sum, evaluated left to right.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define Q19 19

/* Table 1 (Sec. 2.2): components of c_i, i = 0..18. */
static const int CX[Q19] = {0, -1, 0, 0, -1, -1, -1, -1, 0, 0, 1, 0, 0, 1, 1, 1, 1, 0, 0};
static const int CY[Q19] = {0, 0, -1, 0, -1, 1, 0, 0, -1, -1, 0, 1, 0, 1, -1, 0, 0, 1, 1};
static const int CZ[Q19] = {0, 0, 0, -1, 0, 0, -1, 1, -1, 1, 0, 0, 1, 0, 0, 1, -1, 1, -1};

static double weight(int i)
{
    /* w0 = 1/3; w1,2,3,10,11,12 = 1/18; the others 1/36 (Sec. 2.2). */
    if (i == 0) return 1.0 / 3.0;
    if (i == 1 || i == 2 || i == 3 || i == 10 || i == 11 || i == 12) return 1.0 / 18.0;
    return 1.0 / 36.0;
}

/* Opposite direction, found by search over the table (not by formula). */
static int opposite_search(int i)
{
    for (int j = 0; j < Q19; ++j)
        if (CX[j] == -CX[i] && CY[j] == -CY[i] && CZ[j] == -CZ[i]) return j;
    return -1;
}

static int OPP[Q19];
static int opp_ready = 0;

static int opposite(int i)
{
    if (!opp_ready) {
#pragma omp critical(orc_opp)
        {
            if (!opp_ready) {
                for (int j = 0; j < Q19; ++j) OPP[j] = opposite_search(j);
                opp_ready = 1;
            }
        }
    }
    return OPP[i];
}

static int wrap(int a, int n) { return ((a % n) + n) % n; }

static double min_image(double d, double L)
{
    if (d > 0.5 * L) d -= L;
    else if (d < -0.5 * L) d += L;
    return d;
}

void orc_tables(int *c, double *w, int *opp)
{
    for (int i = 0; i < Q19; ++i) {
        c[3 * i + 0] = CX[i];
        c[3 * i + 1] = CY[i];
        c[3 * i + 2] = CZ[i];
        w[i] = weight(i);
        opp[i] = opposite(i);
    }
}

/* Discrete equilibrium, eq. (Equilibre_Maxwell_Boltzmann) with c_s^2 = 1/3:
 * f_i = rho w_i [1 + c.u/cs2 - u.u/(2 cs2) + (c.u)^2/(2 cs2^2)]. */
void orc_equilibrium(double rho, double ux, double uy, double uz, double *feq)
{
    const double cs2 = 1.0 / 3.0;
    double uu = ux * ux + uy * uy + uz * uz;
    for (int i = 0; i < Q19; ++i) {
        double cu = CX[i] * ux + CY[i] * uy + CZ[i] * uz;
        feq[i] = rho * weight(i) * (1.0 + cu / cs2 - uu / (2.0 * cs2) + cu * cu / (2.0 * cs2 * cs2));
    }
}

/* Smagorinsky relaxation time (Sec. 2.2): tau* = tau0 + tau_t with
 * tau_t = [sqrt(tau0^2 + 2 sqrt2 C^2 (rho cs^4)^-1 sqrt(Q)) - tau0] / 2,
 * Q = Pi_ab Pi_ab, filter length and time step 1. */
double orc_relaxation_time(double tau0, double C, double rho, double Q)
{
    const double cs2 = 1.0 / 3.0;
    double tau_t = 0.5 * (sqrt(tau0 * tau0 + 2.0 * sqrt(2.0) * C * C * sqrt(Q) / (rho * cs2 * cs2)) - tau0);
    return tau0 + tau_t;
}

/* Owner map: wall voxels first (walls take precedence), then each sphere
 * claims the nodes p with |p - X|^2 <= R^2 (minimum image) not already
 * claimed, so the lowest sphere index wins an overlap. */
int orc_owner_map(const int *dims, const uint8_t *wall, int n_walls, int nb,
                  const double *X, const double *R, int32_t *owner)
{
    const int nx = dims[0], ny = dims[1], nz = dims[2];
    const long N = (long)nx * ny * nz;
    for (long n = 0; n < N; ++n) {
        int w = wall ? wall[n] : 0;
        if (w > n_walls) return -1;
        owner[n] = w > 0 ? w - 1 : -1;
    }
    for (int b = 0; b < nb; ++b) {
        double cx = X[3 * b], cy = X[3 * b + 1], cz = X[3 * b + 2], r = R[b];
        int x0 = (int)ceil(cx - r), x1 = (int)floor(cx + r);
        int y0 = (int)ceil(cy - r), y1 = (int)floor(cy + r);
        int z0 = (int)ceil(cz - r), z1 = (int)floor(cz + r);
        for (int k = z0; k <= z1; ++k)
            for (int j = y0; j <= y1; ++j)
                for (int i = x0; i <= x1; ++i) {
                    int px = wrap(i, nx), py = wrap(j, ny), pz = wrap(k, nz);
                    double dx = min_image((double)px - cx, nx);
                    double dy = min_image((double)py - cy, ny);
                    double dz = min_image((double)pz - cz, nz);
                    double d2 = dx * dx + dy * dy + dz * dz;
                    if (d2 <= r * r) {
                        long n = px + (long)nx * (py + (long)ny * pz);
                        if (owner[n] < 0) owner[n] = n_walls + b;
                    }
                }
    }
    return 0;
}

typedef struct {
    int nb;
    const double *X, *V, *W, *R;  /* sphere centre, velocity, angular velocity, radius */
    int n_walls;
    const double *Uw, *Ref;        /* wall velocity and torque reference */
} bodies_t;

/* Velocity of the solid that owns node (px,py,pz). */
static void solid_velocity(const bodies_t *B, int own, int px, int py, int pz,
                           const int *dims, double *u)
{
    if (own < B->n_walls) {
        u[0] = B->Uw[3 * own];
        u[1] = B->Uw[3 * own + 1];
        u[2] = B->Uw[3 * own + 2];
        return;
    }
    int b = own - B->n_walls;
    double r0 = min_image(px - B->X[3 * b], dims[0]);
    double r1 = min_image(py - B->X[3 * b + 1], dims[1]);
    double r2 = min_image(pz - B->X[3 * b + 2], dims[2]);
    const double *v = B->V + 3 * b, *w = B->W + 3 * b;
    u[0] = v[0] + (w[1] * r2 - w[2] * r1);
    u[1] = v[1] + (w[2] * r0 - w[0] * r2);
    u[2] = v[2] + (w[0] * r1 - w[1] * r0);
}

/*
 * Streaming and boundary stage of step n.
 *   P        : state after step n-1 (post-collision), [19][N]
 *   own_prev : owner map of step n-1, own_cur: owner map of step n
 *   Bp, Bc   : bodies of step n-1 and of step n
 * Output f  : post-streaming, pre-collision populations at fluid nodes of
 *             step n (solid nodes left untouched); F, T: (nb + W) x 3 force
 *             and torque on each body (spheres first, then walls).
 * halfway != 0 puts every boundary at the link midpoint (q = 1/2).
 */
int orc_stream(const int *dims, const double *prm, int halfway,
               const double *P, const int32_t *own_prev, const int32_t *own_cur,
               int nb_prev, const double *Xp, const double *Vp, const double *Wp, const double *Rp,
               int nb, const double *X, const double *V, const double *W, const double *R,
               int n_walls, const double *Uw, const double *Ref, int zieb_z,
               double *f, double *F, double *T)
{
    const int nx = dims[0], ny = dims[1], nz = dims[2];
    const long N = (long)nx * ny * nz;
    const double rho0 = prm[2];
    bodies_t Bp = {nb_prev, Xp, Vp, Wp, Rp, n_walls, Uw, Ref};
    bodies_t Bc = {nb, X, V, W, R, n_walls, Uw, Ref};
    const int nbt = nb + n_walls;

    /* P-hat: the state, except that every node that was solid at step n-1
     * carries the equilibrium at the reference density and its solid
     * velocity of step n-1 (Sec. 2.3: solid-side populations are a Maxwell
     * equilibrium at the solid velocity). */
    double *Ph = (double *)malloc(sizeof(double) * Q19 * N);
    if (!Ph) return -2;
    memcpy(Ph, P, sizeof(double) * Q19 * N);
    for (long n = 0; n < N; ++n) {
        if (own_prev[n] < 0) continue;
        int px = n % nx, py = (n / nx) % ny, pz = n / ((long)nx * ny);
        double us[3], fe[Q19];
        solid_velocity(&Bp, own_prev[n], px, py, pz, dims, us);
        orc_equilibrium(rho0, us[0], us[1], us[2], fe);
        for (int i = 0; i < Q19; ++i) Ph[i * N + n] = fe[i];
    }

    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    double *acc = (double *)calloc((size_t)nthreads * (nbt > 0 ? nbt : 1) * 6, sizeof(double));
    if (!acc) { free(Ph); return -2; }

#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z) {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *my = acc + (size_t)tid * nbt * 6;
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long n = x + (long)nx * (y + (long)ny * z);
                if (own_cur[n] >= 0) continue;
                f[n] = Ph[n];  /* rest population stays */
                for (int k = 1; k < Q19; ++k) {
                    int i = opposite(k);  /* population that arrives from x + c_k */
                    /* ZIEB plane (Sec. 2.6): nothing arrives from the virtual
                     * domain below it; orc_zieb fills these directions */
                    if (z == zieb_z && CZ[i] == 1) continue;
                    long ns = wrap(x + CX[k], nx) + (long)nx * (wrap(y + CY[k], ny) + (long)ny * wrap(z + CZ[k], nz));
                    int o = own_cur[ns];
                    if (o < 0) {  /* plain streaming: f_i(x) = P(x - c_i)[i] */
                        f[(long)i * N + n] = Ph[(long)i * N + ns];
                        continue;
                    }
                    /* Boundary link from fluid x towards the solid node x + c_k. */
                    double q, arm[3], uw[3];
                    if (o < n_walls) {
                        q = 0.5;
                        arm[0] = x + 0.5 * CX[k] - Ref[3 * o];
                        arm[1] = y + 0.5 * CY[k] - Ref[3 * o + 1];
                        arm[2] = z + 0.5 * CZ[k] - Ref[3 * o + 2];
                        uw[0] = Uw[3 * o]; uw[1] = Uw[3 * o + 1]; uw[2] = Uw[3 * o + 2];
                    } else {
                        int b = o - n_walls;
                        double d[3] = {min_image(x - X[3 * b], nx), min_image(y - X[3 * b + 1], ny),
                                       min_image(z - X[3 * b + 2], nz)};
                        double c[3] = {CX[k], CY[k], CZ[k]};
                        if (halfway) {
                            q = 0.5;
                        } else {
                            /* q: fraction of the link inside the fluid, the
                             * smaller root in (0,1] of |d + q c|^2 = R^2. */
                            double a = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
                            double bb = d[0] * c[0] + d[1] * c[1] + d[2] * c[2];
                            double cc = d[0] * d[0] + d[1] * d[1] + d[2] * d[2] - R[b] * R[b];
                            double disc = bb * bb - a * cc;
                            if (disc < 0.0) disc = 0.0;
                            q = (-bb - sqrt(disc)) / a;
                            if (q > 1.0) q = 1.0;
                            if (q < 0.0) q = 0.0;
                        }
                        for (int a = 0; a < 3; ++a) arm[a] = d[a] + q * c[a];
                        const double *v = V + 3 * b, *w = W + 3 * b;
                        uw[0] = v[0] + (w[1] * arm[2] - w[2] * arm[1]);
                        uw[1] = v[1] + (w[2] * arm[0] - w[0] * arm[2]);
                        uw[2] = v[2] + (w[0] * arm[1] - w[1] * arm[0]);
                    }
                    /* moving-boundary term along the reflected direction i */
                    double ciu = CX[i] * uw[0] + CY[i] * uw[1] + CZ[i] * uw[2];
                    double wk = weight(k);
                    double fk_x = Ph[(long)k * N + n];
                    double fi;
                    if (q < 0.5) {
                        long nm = wrap(x - CX[k], nx) + (long)nx * (wrap(y - CY[k], ny) + (long)ny * wrap(z - CZ[k], nz));
                        if (own_cur[nm] < 0)
                            fi = 2.0 * q * fk_x + (1.0 - 2.0 * q) * Ph[(long)k * N + nm] + 6.0 * wk * rho0 * ciu;
                        else  /* no fluid node behind x: plain bounce-back */
                            fi = fk_x + 6.0 * wk * rho0 * ciu;
                    } else {
                        fi = fk_x / (2.0 * q) + (2.0 * q - 1.0) / (2.0 * q) * Ph[(long)i * N + n]
                             + 3.0 / q * wk * rho0 * ciu;
                    }
                    f[(long)i * N + n] = fi;
                    /* momentum carried into the body along c_k by this link */
                    double m = fk_x + fi;
                    int slot = o < n_walls ? nb + o : o - n_walls;
                    double mc[3] = {m * CX[k], m * CY[k], m * CZ[k]};
                    double *s = my + 6 * slot;
                    s[0] += mc[0];
                    s[1] += mc[1];
                    s[2] += mc[2];
                    s[3] += arm[1] * mc[2] - arm[2] * mc[1];
                    s[4] += arm[2] * mc[0] - arm[0] * mc[2];
                    s[5] += arm[0] * mc[1] - arm[1] * mc[0];
                }
            }
    }
    for (int s = 0; s < nbt; ++s)
        for (int a = 0; a < 3; ++a) {
            double fs = 0.0, ts = 0.0;
            for (int t = 0; t < nthreads; ++t) {
                fs += acc[((size_t)t * nbt + s) * 6 + a];
                ts += acc[((size_t)t * nbt + s) * 6 + 3 + a];
            }
            F[3 * s + a] = fs;
            T[3 * s + a] = ts;
        }
    free(acc);
    free(Ph);
    return 0;
}

/*
 * Zoom-in with Effective Boundaries (Sec. 2.6) at the plane z = zs, fed from
 * a virtual cylinder below it (directions with c_z = +1 are the unknowns).
 *
 * orc_zieb_inflow: the mean in-flowing velocity v_f, the z-velocity of the
 * state P (u = (sum P c - F/2)/rho) averaged over the plane's fluid nodes;
 * also their mean density.
 *
 * orc_zieb_density: eq. (ZIEBdesity8), the explicit update of the density in
 * the virtual cylinder from the piston velocity vp, v_f, the piston area A
 * and the remaining cylinder volume V0 - A Hp (time step 1).
 *
 * orc_zieb: applied to the streamed populations f of the plane's fluid nodes.
 * The unknown directions were not received (orc_stream skips them), so they
 * keep the node's own values P(x_S); with rho* the sum of the populations,
 * f_12 becomes rho_next - (rho* - f_12) (eq. ZIEBdesity9), u = sum f c /
 * rho_next, and every population is set to the equilibrium at (rho_next, u).
 */
int orc_zieb_inflow(const int *dims, const double *prm, const int32_t *own, const double *P, int zs,
                    double *out)
{
    const int nx = dims[0], ny = dims[1];
    const long N = (long)nx * ny * dims[2];
    double su = 0.0, sr = 0.0;
    long cnt = 0;
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            long n = x + (long)nx * (y + (long)ny * zs);
            if (own[n] >= 0) continue;
            double r = 0.0, jz = 0.0;
            for (int i = 0; i < Q19; ++i) {
                r += P[(long)i * N + n];
                jz += CZ[i] * P[(long)i * N + n];
            }
            su += (jz - 0.5 * prm[5]) / r;
            sr += r;
            ++cnt;
        }
    out[0] = cnt ? su / cnt : 0.0;
    out[1] = cnt ? sr / cnt : 0.0;
    return (int)cnt;
}

double orc_zieb_density(double rho, double vp, double vf, double area, double volume, double Hp)
{
    return rho * exp((vp * area - vf * area) / (volume - area * Hp));
}

int orc_zieb(const int *dims, int zs, double rho_next, const int32_t *own, const double *P, double *f)
{
    const int nx = dims[0], ny = dims[1];
    const long N = (long)nx * ny * dims[2];
    const int i12 = 12;  /* (0, 0, 1): streams into the domain normal to the interface */
    for (int y = 0; y < ny; ++y)
        for (int x = 0; x < nx; ++x) {
            long n = x + (long)nx * (y + (long)ny * zs);
            if (own[n] >= 0) continue;
            for (int i = 0; i < Q19; ++i)
                if (CZ[i] == 1) f[(long)i * N + n] = P[(long)i * N + n];
            double rs = 0.0;
            for (int i = 0; i < Q19; ++i) rs += f[(long)i * N + n];
            f[(long)i12 * N + n] = rho_next - (rs - f[(long)i12 * N + n]);
            double j[3] = {0.0, 0.0, 0.0};
            for (int i = 0; i < Q19; ++i) {
                j[0] += CX[i] * f[(long)i * N + n];
                j[1] += CY[i] * f[(long)i * N + n];
                j[2] += CZ[i] * f[(long)i * N + n];
            }
            double fe[Q19];
            orc_equilibrium(rho_next, j[0] / rho_next, j[1] / rho_next, j[2] / rho_next, fe);
            for (int i = 0; i < Q19; ++i) f[(long)i * N + n] = fe[i];
        }
    return 0;
}

/*
 * Collision stage of step n: at fluid nodes, moments -> equilibrium ->
 * Smagorinsky tau* -> BGK with the Guo source; at solid nodes, the
 * equilibrium at the reference density and the solid velocity of step n.
 * prm = {tau0, C, rho0, Fx, Fy, Fz}.  Writes Pout [19][N].
 */
int orc_collide(const int *dims, const double *prm, const int32_t *own,
                int nb, const double *X, const double *V, const double *W, const double *R,
                int n_walls, const double *Uw, const double *Ref,
                const double *f, double *Pout)
{
    const int nx = dims[0], ny = dims[1], nz = dims[2];
    const long N = (long)nx * ny * nz;
    const double tau0 = prm[0], C = prm[1], rho0 = prm[2];
    const double Fb[3] = {prm[3], prm[4], prm[5]};
    bodies_t B = {nb, X, V, W, R, n_walls, Uw, Ref};

#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long n = x + (long)nx * (y + (long)ny * z);
                double fe[Q19];
                if (own[n] >= 0) {
                    double us[3];
                    solid_velocity(&B, own[n], x, y, z, dims, us);
                    orc_equilibrium(rho0, us[0], us[1], us[2], fe);
                    for (int i = 0; i < Q19; ++i) Pout[(long)i * N + n] = fe[i];
                    continue;
                }
                double fi[Q19];
                for (int i = 0; i < Q19; ++i) fi[i] = f[(long)i * N + n];
                /* density and momentum, eqs. (dens) and (momentum) */
                double rho = 0.0, j[3] = {0.0, 0.0, 0.0};
                for (int i = 0; i < Q19; ++i) {
                    rho += fi[i];
                    j[0] += fi[i] * CX[i];
                    j[1] += fi[i] * CY[i];
                    j[2] += fi[i] * CZ[i];
                }
                double u[3];
                for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * Fb[a]) / rho;
                orc_equilibrium(rho, u[0], u[1], u[2], fe);
                /* second moment of the non-equilibrium part */
                double Pi[3][3] = {{0}};
                for (int i = 0; i < Q19; ++i) {
                    int c[3] = {CX[i], CY[i], CZ[i]};
                    for (int a = 0; a < 3; ++a)
                        for (int b = 0; b < 3; ++b) Pi[a][b] += c[a] * c[b] * (fi[i] - fe[i]);
                }
                double Qn = 0.0;
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) Qn += Pi[a][b] * Pi[a][b];
                double ts = orc_relaxation_time(tau0, C, rho, Qn);
                for (int i = 0; i < Q19; ++i) {
                    int c[3] = {CX[i], CY[i], CZ[i]};
                    double cu = c[0] * u[0] + c[1] * u[1] + c[2] * u[2];
                    double src = 0.0;
                    for (int a = 0; a < 3; ++a) src += (3.0 * (c[a] - u[a]) + 9.0 * cu * c[a]) * Fb[a];
                    Pout[(long)i * N + n] = fi[i] - (fi[i] - fe[i]) / ts + (1.0 - 0.5 / ts) * weight(i) * src;
                }
            }
    return 0;
}

/* Initial state: equilibrium of (rho, u) at fluid nodes, equilibrium at the
 * reference density and the solid velocity at solid nodes.  rho, u may be
 * NULL (rho0, 0); u is component-major [3][N]. */
int orc_init(const int *dims, double rho0, const int32_t *own,
             int nb, const double *X, const double *V, const double *W, const double *R,
             int n_walls, const double *Uw, const double *Ref,
             const double *rho, const double *u, double *P)
{
    const long N = (long)dims[0] * dims[1] * dims[2];
    bodies_t B = {nb, X, V, W, R, n_walls, Uw, Ref};
    for (long n = 0; n < N; ++n) {
        double fe[Q19];
        int x = n % dims[0], y = (n / dims[0]) % dims[1], z = n / ((long)dims[0] * dims[1]);
        if (own[n] >= 0) {
            double us[3];
            solid_velocity(&B, own[n], x, y, z, dims, us);
            orc_equilibrium(rho0, us[0], us[1], us[2], fe);
        } else {
            double r = rho ? rho[n] : rho0;
            double ux = u ? u[n] : 0.0, uy = u ? u[N + n] : 0.0, uz = u ? u[2 * N + n] : 0.0;
            orc_equilibrium(r, ux, uy, uz, fe);
        }
        for (int i = 0; i < Q19; ++i) P[(long)i * N + n] = fe[i];
    }
    return 0;
}

/* Density and velocity of a post-collision state at fluid nodes.  The
 * collision adds exactly F to the momentum (Guo source), so the velocity
 * that step's collision used, u = (sum f_pre c + F/2)/rho, is
 * (sum P c - F/2)/rho in terms of the post-collision P; the density is
 * unchanged by the collision.  Solid nodes report rho0 and their solid
 * velocity. */
int orc_macro(const int *dims, const double *prm, const int32_t *own,
              int nb, const double *X, const double *V, const double *W, const double *R,
              int n_walls, const double *Uw, const double *Ref,
              const double *P, double *rho, double *u)
{
    const long N = (long)dims[0] * dims[1] * dims[2];
    const double rho0 = prm[2];
    bodies_t B = {nb, X, V, W, R, n_walls, Uw, Ref};
    for (long n = 0; n < N; ++n) {
        int x = n % dims[0], y = (n / dims[0]) % dims[1], z = n / ((long)dims[0] * dims[1]);
        if (own[n] >= 0) {
            double us[3];
            solid_velocity(&B, own[n], x, y, z, dims, us);
            rho[n] = rho0;
            u[n] = us[0]; u[N + n] = us[1]; u[2 * N + n] = us[2];
            continue;
        }
        double r = 0.0, j[3] = {0, 0, 0};
        for (int i = 0; i < Q19; ++i) {
            double v = P[(long)i * N + n];
            r += v;
            j[0] += v * CX[i]; j[1] += v * CY[i]; j[2] += v * CZ[i];
        }
        rho[n] = r;
        for (int a = 0; a < 3; ++a) u[(long)a * N + n] = (j[a] - 0.5 * prm[3 + a]) / r;
    }
    return 0;
}

int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
