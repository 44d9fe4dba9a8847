/*
 * mpt_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU reference of the per-particle time step of a
 * Lagrangian transport model (the "chemistry-physics processing" modules of
 * Sec. 3.2: module_advection, module_diffusion_turb, module_diffusion_meso,
 * module_position, module_timesteps), with the random numbers of Sec. 4.3
 * (randoms_t, Listing 6: three normals per parcel and step for turbulent and
 * three for mesoscale diffusion) drawn from a counter-based Philox4x32-10.
 *
 * Only the tests, the smoke check and the CPU-baseline leg of the benchmark
 * may load this library.  It shares no code, header, table or constant with
 * the GPU library: every formula below is written out here on its own.
 *
 * The paper names the modules and says what each does but states no
 * equation; every formula here is a reading, listed with its reason in the
 * design notes:
 *   - locate + quadrilinear interpolation in (lon, lat, p, t); lon periodic
 *     (read_met_periodic, Sec. 3.1), lat and p clamped, weight linear in p;
 *   - explicit midpoint advection (module_advection, Sec. 3.2);
 *   - Fickian random walk for turbulent diffusion (module_diffusion_turb);
 *   - AR(1) sub-grid wind from the variance of the 16 values of the grid
 *     cell for mesoscale diffusion (module_diffusion_meso; state in `cache`,
 *     Sec. 4.1 data regions);
 *   - pole reflection, lon wrap to [0, 360), p clamp (module_position);
 *   - activity gating: non-finite or not-yet-released parcels are skipped
 *     (module_timesteps, Sec. 4.3);
 *   - unresolved convection (module_convection, Sec. 3.2): where the CAPE at
 *     the parcel reaches a threshold and the parcel is below the equilibrium
 *     level, it is placed at a pressure drawn uniformly between the surface
 *     and the equilibrium level (one uniform per parcel and step, the
 *     `convection` slot of randoms_t, Sec. 4.3);
 *   - sedimentation (module_sedi, Sec. 3.2): Stokes settling of a sphere
 *     with the Cunningham slip correction, air viscosity by Sutherland's law,
 *     converted to pressure with the scale height of the turbulent step.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (no -ffast-math).
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <omp.h>

/* ---- physical constants of the reading (own copies) -------------------- */
#define ORC_PI        3.14159265358979323846
#define ORC_R_EARTH   6371000.0          /* mean Earth radius [m]           */
#define ORC_H0        7000.0             /* scale height for dz -> dp [m]   */
#define ORC_LAT_CAP   89.999             /* cos(lat) floor latitude [deg]   */

#define ORC_G0        9.80665            /* standard gravity [m/s^2]        */
#define ORC_RD        287.058            /* gas constant of dry air [J/kg/K] */

#define ORC_ADVECT 1
#define ORC_TURB   2
#define ORC_MESO   4
#define ORC_CONV   8
#define ORC_SEDI   16

/* Met fields on a regular lon-lat grid with fixed pressure levels.
 * u, v in m/s, w in hPa/s; index ((l*nz + k)*ny + j)*nx + i. */
typedef struct {
    int32_t nx, ny, nz, nt;
    double lon0, dlon, lat0, dlat;
    const double *plev;          /* nz values, hPa, strictly decreasing */
    double t_met0, dt_met;
    const float *u, *v, *w;
    int32_t analytic;            /* 0: gridded winds; 1: solid-body rotation */
    int32_t pad_;
    double an_u0, an_alpha;      /* rotation speed [m/s], axis tilt [rad]   */
    /* convection and sedimentation: temperature [K] as u; CAPE [J/kg],
     * equilibrium-level and surface pressure [hPa] per (l, j, i) */
    const float *temp;
    const float *cape, *pel, *ps;
} orc_met;

typedef struct {
    double dt, t_start;          /* s; step n starts at t_start + n*dt      */
    double turb_dx, turb_dz;     /* m^2/s                                    */
    double meso_fh, meso_fv;     /* dimensionless                            */
    uint64_t seed;
    int32_t flags;               /* ORC_ADVECT | ORC_TURB | ORC_MESO |
                                    ORC_CONV | ORC_SEDI                      */
    int32_t pad_;
    double conv_cape;            /* CAPE threshold [J/kg]                    */
    double sedi_r, sedi_rho;     /* particle radius [m], density [kg/m^3]    */
} orc_ctl;

/* ======================================================================= */
/* Grid cell location (periodic lon, clamped lat, level bracket, time pair) */
/* ======================================================================= */

typedef struct {
    int i0, i1, j, k, l;
    double fx, fy, fz, ft;
} orc_loc;

static void orc_locate(const orc_met *m, double lon, double lat, double p, double t, orc_loc *L)
{
    /* longitude: bring into [lon0, lon0+360), index i with wrap */
    double lam = lon - 360.0 * floor((lon - m->lon0) / 360.0);
    double x = (lam - m->lon0) / m->dlon;
    double xf = floor(x);
    long ii = (long)xf % m->nx;
    if (ii < 0) ii += m->nx;
    L->i0 = (int)ii;
    L->i1 = (int)((ii + 1) % m->nx);
    L->fx = x - xf;

    /* latitude: clamp to the grid's range, bottom row index <= ny-2 */
    double lat_hi = m->lat0 + (m->ny - 1) * m->dlat;
    double phi = lat < m->lat0 ? m->lat0 : (lat > lat_hi ? lat_hi : lat);
    double y = (phi - m->lat0) / m->dlat;
    int jj = (int)floor(y);
    if (jj > m->ny - 2) jj = m->ny - 2;
    if (jj < 0) jj = 0;
    L->j = jj;
    L->fy = y - jj;

    /* pressure: clamp to [plev[nz-1], plev[0]]; k = largest index <= nz-2
     * with plev[k] >= p; weight linear in p */
    double ptop = m->plev[m->nz - 1], pbot = m->plev[0];
    double pc = p < ptop ? ptop : (p > pbot ? pbot : p);
    int kk = m->nz - 2;
    while (kk > 0 && m->plev[kk] < pc) kk--;
    L->k = kk;
    L->fz = (m->plev[kk] - pc) / (m->plev[kk] - m->plev[kk + 1]);

    /* time: bracketing pair l, l+1 of the resident levels */
    double tl = floor((t - m->t_met0) / m->dt_met);
    int ll = (int)tl;
    if (tl < 0) ll = 0;
    if (ll > m->nt - 2) ll = m->nt - 2;
    L->l = ll;
    L->ft = (t - (m->t_met0 + ll * m->dt_met)) / m->dt_met;
}

static size_t orc_idx(const orc_met *m, int l, int k, int j, int i)
{
    return (((size_t)l * m->nz + k) * m->ny + j) * (size_t)m->nx + i;
}

static double orc_lerp(double a, double b, double f) { return (1.0 - f) * a + f * b; }

/* Quadrilinear interpolation of one variable: along lon, then lat, then p,
 * at both time levels, then in time. */
static double orc_interp_var(const orc_met *m, const float *f, const orc_loc *L)
{
    double lev[2];
    for (int dl = 0; dl < 2; ++dl) {
        double zk[2];
        for (int dk = 0; dk < 2; ++dk) {
            double yj[2];
            for (int dj = 0; dj < 2; ++dj) {
                double a = f[orc_idx(m, L->l + dl, L->k + dk, L->j + dj, L->i0)];
                double b = f[orc_idx(m, L->l + dl, L->k + dk, L->j + dj, L->i1)];
                yj[dj] = orc_lerp(a, b, L->fx);
            }
            zk[dk] = orc_lerp(yj[0], yj[1], L->fy);
        }
        lev[dl] = orc_lerp(zk[0], zk[1], L->fz);
    }
    return orc_lerp(lev[0], lev[1], L->ft);
}

/* Tilted solid-body rotation (Williamson et al. 1992, test case 1):
 * u = U0 (cos(lat) cos(a) + sin(lat) cos(lon) sin(a)), v = -U0 sin(lon) sin(a). */
static void orc_wind_analytic(const orc_met *m, double lon, double lat, double uvw[3])
{
    double d2r = ORC_PI / 180.0;
    double la = lon * d2r, ph = lat * d2r, a = m->an_alpha;
    uvw[0] = m->an_u0 * (cos(ph) * cos(a) + sin(ph) * cos(la) * sin(a));
    uvw[1] = -m->an_u0 * sin(la) * sin(a);
    uvw[2] = 0.0;
}

static void orc_wind(const orc_met *m, double lon, double lat, double p, double t, double uvw[3])
{
    if (m->analytic) {
        orc_wind_analytic(m, lon, lat, uvw);
        return;
    }
    orc_loc L;
    orc_locate(m, lon, lat, p, t, &L);
    uvw[0] = orc_interp_var(m, m->u, &L);
    uvw[1] = orc_interp_var(m, m->v, &L);
    uvw[2] = orc_interp_var(m, m->w, &L);
}

/* ======================================================================= */
/* Unit conversions                                                        */
/* ======================================================================= */

static double orc_cos_floor(double lat)
{
    double c = cos(lat * ORC_PI / 180.0);
    double cmin = cos(ORC_LAT_CAP * ORC_PI / 180.0);
    return c > cmin ? c : cmin;
}

/* eastward distance [m] -> degrees of longitude at latitude lat */
static double orc_dx2deg(double dx, double lat)
{
    return dx * 180.0 / (ORC_PI * ORC_R_EARTH * orc_cos_floor(lat));
}

/* northward distance [m] -> degrees of latitude */
static double orc_dy2deg(double dy) { return dy * 180.0 / (ORC_PI * ORC_R_EARTH); }

/* ======================================================================= */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and normals            */
/* ======================================================================= */

static void orc_mulhilo(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo)
{
    uint64_t prod = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(prod >> 32);
    *lo = (uint32_t)prod;
}

void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c[4] = {ctr_in[0], ctr_in[1], ctr_in[2], ctr_in[3]};
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        if (r > 0) {                  /* Weyl sequence key schedule */
            k0 += 0x9E3779B9u;
            k1 += 0xBB67AE85u;
        }
        uint32_t hi0, lo0, hi1, lo1;
        orc_mulhilo(0xD2511F53u, c[0], &hi0, &lo0);
        orc_mulhilo(0xCD9E8D57u, c[2], &hi1, &lo1);
        uint32_t n0 = hi1 ^ c[1] ^ k0;
        uint32_t n2 = hi0 ^ c[3] ^ k1;
        c[0] = n0;
        c[1] = lo1;
        c[2] = n2;
        c[3] = lo0;
    }
    out[0] = c[0]; out[1] = c[1]; out[2] = c[2]; out[3] = c[3];
}

/* 24-bit uniform in (0, 1): ((x >> 8) + 1/2) / 2^24 */
double orc_uniform(uint32_t x) { return ((double)(x >> 8) + 0.5) * (1.0 / 16777216.0); }

/* Three standard normals for (parcel id, step, purpose) by Box-Muller
 * (Box & Muller 1958) on the four uniforms of one Philox block. */
void orc_normals3(uint64_t seed, uint32_t id, uint32_t step, uint32_t purpose, double xi[3])
{
    uint32_t ctr[4] = {id, step, purpose, 0u};
    uint32_t key[2] = {(uint32_t)(seed & 0xffffffffu), (uint32_t)(seed >> 32)};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    double u0 = orc_uniform(x[0]), u1 = orc_uniform(x[1]);
    double u2 = orc_uniform(x[2]), u3 = orc_uniform(x[3]);
    double r0 = sqrt(-2.0 * log(u0));
    double r1 = sqrt(-2.0 * log(u2));
    xi[0] = r0 * cos(2.0 * ORC_PI * u1);
    xi[1] = r0 * sin(2.0 * ORC_PI * u1);
    xi[2] = r1 * cos(2.0 * ORC_PI * u3);
}

/* ======================================================================= */
/* Modules                                                                  */
/* ======================================================================= */

/* tendency f(x, t) = (u / (R cos lat), v / R, omega) in deg/s, deg/s, hPa/s */
static void orc_tendency(const orc_met *m, double lon, double lat, double p, double t, double d[3])
{
    double uvw[3];
    orc_wind(m, lon, lat, p, t, uvw);
    d[0] = orc_dx2deg(uvw[0], lat);
    d[1] = orc_dy2deg(uvw[1]);
    d[2] = uvw[2];
}

/* explicit midpoint: x_mid = x + dt/2 f(x, t); x' = x + dt f(x_mid, t + dt/2) */
static void orc_advect(const orc_met *m, double dt, double t, double *lon, double *lat, double *p)
{
    double d0[3], d1[3];
    orc_tendency(m, *lon, *lat, *p, t, d0);
    double lonm = *lon + 0.5 * dt * d0[0];
    double latm = *lat + 0.5 * dt * d0[1];
    double pm = *p + 0.5 * dt * d0[2];
    orc_tendency(m, lonm, latm, pm, t + 0.5 * dt, d1);
    *lon = *lon + dt * d1[0];
    *lat = *lat + dt * d1[1];
    *p = *p + dt * d1[2];
}

/* keep the parcel in the domain: reflect over the poles, wrap lon to
 * [0, 360), clamp p to the level range */
static void orc_position(const orc_met *m, double *lon, double *lat, double *p)
{
    if (*lat > 90.0) {
        *lat = 180.0 - *lat;
        *lon += 180.0;
    } else if (*lat < -90.0) {
        *lat = -180.0 - *lat;
        *lon += 180.0;
    }
    double x = fmod(*lon, 360.0);
    if (x < 0.0) x += 360.0;
    if (x >= 360.0) x = 0.0;
    *lon = x;
    double ptop = m->plev[m->nz - 1], pbot = m->plev[0];
    if (*p < ptop) *p = ptop;
    if (*p > pbot) *p = pbot;
}

/* Fickian random walk: horizontal sigma sqrt(2 Dx dt), vertical
 * sqrt(2 Dz dt) metres, converted with dp = -p/H0 dz */
static void orc_turb(const orc_ctl *c, const double xi[3], double *lon, double *lat, double *p)
{
    double sh = sqrt(2.0 * c->turb_dx * c->dt);
    double sz = sqrt(2.0 * c->turb_dz * c->dt);
    double dlon = orc_dx2deg(sh * xi[0], *lat);
    double dlat = orc_dy2deg(sh * xi[1]);
    double dp = -(sz * xi[2]) * (*p) / ORC_H0;
    *lon += dlon;
    *lat += dlat;
    *p += dp;
}

/* standard deviation (two-pass, population) of the 16 values of one
 * variable on the 8 cell corners at the 2 time levels */
static double orc_cell_sigma(const orc_met *m, const float *f, const orc_loc *L)
{
    double x[16];
    int n = 0;
    for (int dl = 0; dl < 2; ++dl)
        for (int dk = 0; dk < 2; ++dk)
            for (int dj = 0; dj < 2; ++dj) {
                x[n++] = f[orc_idx(m, L->l + dl, L->k + dk, L->j + dj, L->i0)];
                x[n++] = f[orc_idx(m, L->l + dl, L->k + dk, L->j + dj, L->i1)];
            }
    double mean = 0.0;
    for (int q = 0; q < 16; ++q) mean += x[q];
    mean /= 16.0;
    double var = 0.0;
    for (int q = 0; q < 16; ++q) var += (x[q] - mean) * (x[q] - mean);
    var /= 16.0;
    return sqrt(var > 0.0 ? var : 0.0);
}

/* AR(1) sub-grid wind: w' <- r w' + sqrt(1-r^2) f sigma xi,
 * r = 1 - 2 dt / dt_met (>= 0); then displace by w' dt */
static void orc_meso(const orc_met *m, const orc_ctl *c, double t_mid, const double xi[3],
                     double *lon, double *lat, double *p, double *up, double *vp, double *wp)
{
    orc_loc L;
    orc_locate(m, *lon, *lat, *p, t_mid, &L);
    double su = orc_cell_sigma(m, m->u, &L);
    double sv = orc_cell_sigma(m, m->v, &L);
    double sw = orc_cell_sigma(m, m->w, &L);
    double r = 1.0 - 2.0 * c->dt / m->dt_met;
    if (r < 0.0) r = 0.0;
    double rs = sqrt(1.0 - r * r);
    *up = r * (*up) + rs * c->meso_fh * su * xi[0];
    *vp = r * (*vp) + rs * c->meso_fh * sv * xi[1];
    *wp = r * (*wp) + rs * c->meso_fv * sw * xi[2];
    double dlon = orc_dx2deg((*up) * c->dt, *lat);
    double dlat = orc_dy2deg((*vp) * c->dt);
    double dp = (*wp) * c->dt;
    *lon += dlon;
    *lat += dlat;
    *p += dp;
}

/* Bilinear in (lon, lat) at both time levels, then linear in time, of a
 * field with one value per (l, j, i). */
static double orc_interp_2d(const orc_met *m, const float *f, const orc_loc *L)
{
    double lev[2];
    for (int dl = 0; dl < 2; ++dl) {
        size_t r0 = ((size_t)(L->l + dl) * m->ny + L->j) * (size_t)m->nx;
        size_t r1 = r0 + (size_t)m->nx;
        double y0 = orc_lerp(f[r0 + L->i0], f[r0 + L->i1], L->fx);
        double y1 = orc_lerp(f[r1 + L->i0], f[r1 + L->i1], L->fx);
        lev[dl] = orc_lerp(y0, y1, L->fy);
    }
    return orc_lerp(lev[0], lev[1], L->ft);
}

/* Unresolved convection: CAPE, equilibrium level pel and surface pressure ps
 * at the parcel (time t_mid); where CAPE >= the threshold and the parcel is
 * below the equilibrium level (p > pel), the new pressure is
 * ps + (pel - ps) u with u uniform on (0, 1): equal pressure intervals hold
 * equal air mass, so the column between surface and equilibrium level is
 * mixed by mass.  u is the first word of the Philox block of counter
 * (id, step, 5, 0). */
static void orc_convection(const orc_met *m, const orc_ctl *c, uint32_t id, uint32_t step,
                           double t_mid, double lon, double lat, double *p)
{
    orc_loc L;
    orc_locate(m, lon, lat, *p, t_mid, &L);
    double cape = orc_interp_2d(m, m->cape, &L);
    double pel = orc_interp_2d(m, m->pel, &L);
    double ps = orc_interp_2d(m, m->ps, &L);
    if (!(cape >= c->conv_cape) || !(*p > pel)) return;
    uint32_t ctr[4] = {id, step, 5u, 0u};
    uint32_t key[2] = {(uint32_t)c->seed, (uint32_t)(c->seed >> 32)};
    uint32_t x[4];
    orc_philox4x32_10(ctr, key, x);
    *p = ps + (pel - ps) * orc_uniform(x[0]);
}

/* Settling velocity [m/s] of a sphere of radius r [m] and density rho_p
 * [kg/m^3] in air at pressure p [hPa] and temperature T [K]: Stokes drag
 * with the Cunningham slip correction
 *   v = 2 r^2 (rho_p - rho) g Cc / (9 eta),
 *   Cc = 1 + Kn (1.257 + 0.4 exp(-1.1 / Kn)),  Kn = lambda / r,
 *   lambda = 2 eta / (rho vbar),  vbar = sqrt(8 R_d T / pi),
 *   rho = 100 p / (R_d T),  eta = 1.458e-6 T^1.5 / (T + 110.4)  (Sutherland). */
double orc_settling_velocity(double r, double rho_p, double p, double T)
{
    double rho = 100.0 * p / (ORC_RD * T);
    double eta = 1.458e-6 * T * sqrt(T) / (T + 110.4);
    double vbar = sqrt(8.0 * ORC_RD * T / ORC_PI);
    double lambda = 2.0 * eta / (rho * vbar);
    double kn = lambda / r;
    double cc = 1.0 + kn * (1.257 + 0.4 * exp(-1.1 / kn));
    return 2.0 * r * r * (rho_p - rho) * ORC_G0 * cc / (9.0 * eta);
}

/* Sedimentation: the parcel sinks v dt metres; dp = p v dt / H0 (the
 * scale-height conversion of the turbulent step).  T at the parcel, time
 * t_mid. */
static void orc_sedi(const orc_met *m, const orc_ctl *c, double t_mid, double lon, double lat,
                     double *p)
{
    orc_loc L;
    orc_locate(m, lon, lat, *p, t_mid, &L);
    double T = orc_interp_var(m, m->temp, &L);
    double v = orc_settling_velocity(c->sedi_r, c->sedi_rho, *p, T);
    *p += (*p) * v * c->dt / ORC_H0;
}

/* one time step of one parcel, in the order advection, position,
 * turbulent diffusion, mesoscale diffusion, position, convection,
 * sedimentation, position */
static void orc_step_one(const orc_met *m, const orc_ctl *c, uint32_t step, uint32_t id,
                         int32_t release, double *lon, double *lat, double *p,
                         double *up, double *vp, double *wp)
{
    if (!isfinite(*lon) || !isfinite(*lat) || !isfinite(*p)) return;
    if ((int64_t)step < (int64_t)release) return;
    double t = c->t_start + (double)step * c->dt;
    if (c->flags & ORC_ADVECT) {
        orc_advect(m, c->dt, t, lon, lat, p);
        orc_position(m, lon, lat, p);
    }
    if (c->flags & (ORC_TURB | ORC_MESO)) {
        double xi[3];
        if (c->flags & ORC_TURB) {
            orc_normals3(c->seed, id, step, 0u, xi);
            orc_turb(c, xi, lon, lat, p);
        }
        if (c->flags & ORC_MESO) {
            orc_normals3(c->seed, id, step, 1u, xi);
            orc_meso(m, c, t + 0.5 * c->dt, xi, lon, lat, p, up, vp, wp);
        }
        orc_position(m, lon, lat, p);
    }
    if (c->flags & (ORC_CONV | ORC_SEDI)) {
        if (c->flags & ORC_CONV) orc_convection(m, c, id, step, t + 0.5 * c->dt, *lon, *lat, p);
        if (c->flags & ORC_SEDI) orc_sedi(m, c, t + 0.5 * c->dt, *lon, *lat, p);
        orc_position(m, lon, lat, p);
    }
}

/* ======================================================================= */
/* Exported entry points                                                    */
/* ======================================================================= */

/* Run steps step0 .. step0+nsteps-1 on n parcels in place.  release may be
 * NULL (all active); otherwise a parcel is skipped while step < release[i]. */
void orc_run(const orc_met *m, const orc_ctl *c, int64_t n, double *lon, double *lat, double *p,
             const uint32_t *id, double *up, double *vp, double *wp, const int32_t *release,
             uint32_t step0, int32_t nsteps, int32_t nthreads)
{
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        int32_t rel = release ? release[i] : INT32_MIN;
        for (int32_t s = 0; s < nsteps; ++s)
            orc_step_one(m, c, step0 + (uint32_t)s, id[i], rel, &lon[i], &lat[i], &p[i],
                         &up[i], &vp[i], &wp[i]);
    }
}

/* Interpolated (u, v, w) at n points, time t; out[3*i + var]. */
void orc_interp_many(const orc_met *m, int64_t n, const double *lon, const double *lat,
                     const double *p, double t, double *out)
{
    for (int64_t i = 0; i < n; ++i) orc_wind(m, lon[i], lat[i], p[i], t, &out[3 * i]);
}

/* Cell standard deviations (u, v, w) at n points, time t; out[3*i + var]. */
void orc_cell_sigma_many(const orc_met *m, int64_t n, const double *lon, const double *lat,
                         const double *p, double t, double *out)
{
    for (int64_t i = 0; i < n; ++i) {
        orc_loc L;
        orc_locate(m, lon[i], lat[i], p[i], t, &L);
        out[3 * i + 0] = orc_cell_sigma(m, m->u, &L);
        out[3 * i + 1] = orc_cell_sigma(m, m->v, &L);
        out[3 * i + 2] = orc_cell_sigma(m, m->w, &L);
    }
}

/* Cell indices (i0, j, k, l) at n points; out[4*i + q]. */
void orc_locate_many(const orc_met *m, int64_t n, const double *lon, const double *lat,
                     const double *p, double t, int32_t *out_idx, double *out_frac)
{
    for (int64_t i = 0; i < n; ++i) {
        orc_loc L;
        orc_locate(m, lon[i], lat[i], p[i], t, &L);
        out_idx[4 * i + 0] = L.i0;
        out_idx[4 * i + 1] = L.j;
        out_idx[4 * i + 2] = L.k;
        out_idx[4 * i + 3] = L.l;
        out_frac[4 * i + 0] = L.fx;
        out_frac[4 * i + 1] = L.fy;
        out_frac[4 * i + 2] = L.fz;
        out_frac[4 * i + 3] = L.ft;
    }
}

/* Position fix on n parcels in place. */
void orc_position_many(const orc_met *m, int64_t n, double *lon, double *lat, double *p)
{
    for (int64_t i = 0; i < n; ++i) orc_position(m, &lon[i], &lat[i], &p[i]);
}

/* Philox4x32-10 on n counters (4 words each) under one key. */
void orc_philox_many(int64_t n, const uint32_t *ctr, const uint32_t key[2], uint32_t *out)
{
    for (int64_t i = 0; i < n; ++i) orc_philox4x32_10(&ctr[4 * i], key, &out[4 * i]);
}

/* Normals for n ids at one (step, purpose); out[3*i + q]. */
void orc_normals_many(uint64_t seed, int64_t n, const uint32_t *id, uint32_t step, uint32_t purpose,
                      double *out)
{
    for (int64_t i = 0; i < n; ++i) orc_normals3(seed, id[i], step, purpose, &out[3 * i]);
}

/* Grid-box sort key of the cell that holds the position: its 8 x 8 x 4
 * (lon x lat x level) tile, tiles numbered with lon fastest, then lat, then
 * level; then, inside the tile, which half of the tile the cell lies in
 * along level, lat and lon (the upper half counting 4, 2 and 1), so that a
 * tile's 8 half-tiles of 4 x 4 x 2 cells follow each other:
 * key = 8 * tile + half-tile.  Non-finite positions get the key one past the
 * last cell key. */
void orc_tile_keys(const orc_met *m, int64_t n, const double *lon, const double *lat,
                   const double *p, uint32_t *out)
{
    uint32_t ntx = (uint32_t)((m->nx + 7) / 8);
    uint32_t nty = (uint32_t)((m->ny - 1 + 7) / 8);
    uint32_t ntz = (uint32_t)((m->nz - 1 + 3) / 4);
    for (int64_t i = 0; i < n; ++i) {
        if (!isfinite(lon[i]) || !isfinite(lat[i]) || !isfinite(p[i])) {
            out[i] = 8u * ntx * nty * ntz;
            continue;
        }
        orc_loc L;
        orc_locate(m, lon[i], lat[i], p[i], m->t_met0, &L);
        uint32_t tile = ((uint32_t)(L.k / 4) * nty + (uint32_t)(L.j / 8)) * ntx + (uint32_t)(L.i0 / 8);
        uint32_t half = 4u * (uint32_t)(L.k % 4 >= 2) + 2u * (uint32_t)(L.j % 8 >= 4) + (uint32_t)(L.i0 % 8 >= 4);
        out[i] = 8u * tile + half;
    }
}

/* ----------------------------------------------------------------------- */
/* Surrogate inputs and targets (project addition: learned k-step advection) */
/* ----------------------------------------------------------------------- */

/* Quadrilinear value of one variable in the cell shifted by (a, b, c) grid
 * steps from the parcel's cell, with the parcel's own weights: columns wrap,
 * rows and levels are clamped to the grid. */
static double orc_interp_shifted(const orc_met *m, const float *f, const orc_loc *L, int a, int b, int c)
{
    orc_loc S = *L;
    int i0 = (L->i0 + a) % m->nx;
    if (i0 < 0) i0 += m->nx;
    S.i0 = i0;
    S.i1 = (i0 + 1) % m->nx;
    int j = L->j + b;
    S.j = j < 0 ? 0 : (j > m->ny - 2 ? m->ny - 2 : j);
    int k = L->k + c;
    S.k = k < 0 ? 0 : (k > m->nz - 2 ? m->nz - 2 : k);
    return orc_interp_var(m, f, &S);
}

/* The 81 surrogate inputs of n parcels at time t: u, v, w on the 3 x 3 x 3
 * stencil of cells around the parcel's cell (offsets -1, 0, 1 in lon, lat,
 * level), out[81*i + var*27 + (c+1)*9 + (b+1)*3 + (a+1)]. */
void orc_stencil81_many(const orc_met *m, int64_t n, const double *lon, const double *lat,
                        const double *p, double t, double *out)
{
    for (int64_t i = 0; i < n; ++i) {
        orc_loc L;
        orc_locate(m, lon[i], lat[i], p[i], t, &L);
        const float *fld[3] = {m->u, m->v, m->w};
        for (int q = 0; q < 3; ++q)
            for (int c = -1; c <= 1; ++c)
                for (int b = -1; b <= 1; ++b)
                    for (int a = -1; a <= 1; ++a)
                        out[81 * i + q * 27 + (c + 1) * 9 + (b + 1) * 3 + (a + 1)] =
                            orc_interp_shifted(m, fld[q], &L, a, b, c);
    }
}

/* k-step displacement of plain advection (no diffusion) from (lon, lat, p)
 * at step `step0`: east and north distance in km (east measured along the
 * start latitude: dlon * pi R cos(lat0) / 180) and pressure change in hPa;
 * out[3*i + q]. */
void orc_displacement_many(const orc_met *m, const orc_ctl *c, int64_t n, const double *lon,
                           const double *lat, const double *p, uint32_t step0, int32_t k,
                           double *out, int32_t nthreads)
{
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for num_threads(nthreads) schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        double x = lon[i], y = lat[i], z = p[i];
        for (int32_t s = 0; s < k; ++s) {
            double t = c->t_start + (double)(step0 + (uint32_t)s) * c->dt;
            orc_advect(m, c->dt, t, &x, &y, &z);
            orc_position(m, &x, &y, &z);
        }
        double dl = fmod(x - lon[i] + 540.0, 360.0) - 180.0;
        out[3 * i + 0] = dl * ORC_PI * ORC_R_EARTH * orc_cos_floor(lat[i]) / 180.0 / 1000.0;
        out[3 * i + 1] = (y - lat[i]) * ORC_PI * ORC_R_EARTH / 180.0 / 1000.0;
        out[3 * i + 2] = z - p[i];
    }
}

/* ---- gridded output (write_grid, Sec. 3.3; a reading: the paper names the
 * function only).  Box (k, j, i) of a regular grid, index (k*ny + j)*nx + i:
 *   i = floor((lon - lon0) / dlon) mod nx,
 *   j = floor((lat - lat0) / dlat) if 0 <= j < ny; j = ny - 1 when lat equals
 *       the grid's north edge lat0 + ny*dlat; otherwise outside,
 *   k: pedges[k] >= p > pedges[k+1] (edges decreasing), found by walking the
 *       layers; outside if there is none.
 * counts[b] = number of parcels in b, msum[b] = sum of their masses (1 each
 * when mass is NULL), mmr[b] = msum[b] / air mass of b, air mass =
 * R^2 * dlon[rad] * (sin(lat north) - sin(lat south)) * dp[Pa] / g. */
#define ORC_G 9.80665
void orc_grid_output(int64_t n, const double *lon, const double *lat, const double *p,
                     const double *mass, int nx, int ny, int nz, double lon0, double dlon,
                     double lat0, double dlat, const double *pedges, uint32_t *counts,
                     double *msum, double *mmr)
{
  const int64_t nbox = (int64_t)nx * ny * nz;
  for (int64_t b = 0; b < nbox; ++b) { counts[b] = 0; msum[b] = 0.0; }
  for (int64_t q = 0; q < n; ++q) {
    if (!isfinite(lon[q]) || !isfinite(lat[q]) || !isfinite(p[q])) continue;
    int64_t i = (int64_t)floor((lon[q] - lon0) / dlon) % nx;
    if (i < 0) i += nx;
    const double y = floor((lat[q] - lat0) / dlat);
    int64_t j;
    if (y < 0.0) continue;
    if (y >= (double)ny) {
      if (lat[q] != lat0 + ny * dlat) continue;
      j = ny - 1;
    } else {
      j = (int64_t)y;
    }
    int k = -1;
    for (int kk = 0; kk < nz; ++kk)
      if (pedges[kk] >= p[q] && p[q] > pedges[kk + 1]) { k = kk; break; }
    if (k < 0) continue;
    const int64_t b = ((int64_t)k * ny + j) * nx + i;
    counts[b] += 1;
    msum[b] += mass ? mass[q] : 1.0;
  }
  for (int64_t b = 0; b < nbox; ++b) {
    const int64_t k = b / ((int64_t)nx * ny), j = (b / nx) % ny;
    const double s0 = sin((lat0 + j * dlat) * ORC_PI / 180.0);
    const double s1 = sin((lat0 + (j + 1) * dlat) * ORC_PI / 180.0);
    const double air = ORC_R_EARTH * ORC_R_EARTH * (dlon * ORC_PI / 180.0) * (s1 - s0) *
                       (pedges[k] - pedges[k + 1]) * 100.0 / ORC_G;
    mmr[b] = msum[b] / air;
  }
}

/* ---- hybrid model levels to pressure levels (read_met regridding the
 * model-level data, Sec. 3.1; a reading).  Column pressures
 * p_k = a_k + b_k ps (k = 0 lowest, decreasing with k); a target level p
 * between p_k >= p > p_{k+1} gets f_k + (ln p_k - ln p) / (ln p_k - ln p_{k+1})
 * (f_{k+1} - f_k); a target below the lowest or above the highest model level
 * of its column gets that level's value.  FP64, rounded to float. */
void orc_ml_to_pl(int nx, int ny, int nz, const double *plev, int nml, const double *a,
                  const double *b, const float *ps, const float *f, float *out)
{
  const int64_t ncol = (int64_t)nx * ny;
  for (int m = 0; m < nz; ++m)
    for (int64_t col = 0; col < ncol; ++col) {
      const double s = ps[col], p = plev[m];
      double val;
      if (p >= a[0] + b[0] * s) {
        val = f[col];
      } else if (p <= a[nml - 1] + b[nml - 1] * s) {
        val = f[(int64_t)(nml - 1) * ncol + col];
      } else {
        int k = 0;
        while (!(a[k] + b[k] * s >= p && p > a[k + 1] + b[k + 1] * s)) ++k;
        const double pk = a[k] + b[k] * s, pk1 = a[k + 1] + b[k + 1] * s;
        const double f0 = f[(int64_t)k * ncol + col], f1 = f[(int64_t)(k + 1) * ncol + col];
        val = f0 + (log(pk) - log(p)) / (log(pk) - log(pk1)) * (f1 - f0);
      }
      out[(int64_t)m * ncol + col] = (float)val;
    }
}

int orc_max_threads(void) { return omp_get_max_threads(); }
