/*
 * FP64 CPU oracle for the phase-field thermocapillary lattice Boltzmann scheme of
 * L. Wang, K. He and H. Wang, "Phase-field-based lattice Boltzmann model for
 * simulating thermocapillary flows" (arXiv:2306.11320).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow, obviously correct
 * reference that the HIP path is checked against.  Only the tests, the smoke
 * check and the CPU-baseline leg of the benchmark may load it; the product path
 * never does.  It shares no code, header, table or constant with the HIP path.
 *
 * Every step follows the paper's order and notation, two passes per time step:
 *   pass 1: macroscopic fields at every node (phi, T, stencils, F_s, u, p);
 *   pass 2: the three BGK collisions and push streaming with the boundary rules.
 * Compiled with -O2 -ffp-contract=off so no fused multiply-adds change rounding.
 *
 * Lattice units: dx = dt = 1, c = 1, c_s^2 = 1/3 (Sec. 4, preamble).
 *
 * Readings of points where the paper is silent, garbled or self-inconsistent
 * (each is listed with its reason in the design notes of the repository):
 *   - phi_l = -1 (light), phi_h = +1 (heavy); counter term (1-phi^2)/(sqrt2 W),
 *     equilibrium profile tanh(d/(sqrt2 W)) (Sec. 2, Eq. 5);
 *   - D2Q9 weights 4/9, 1/9, 1/36 (the printed 4/9 for i=1..4 cannot sum to 1);
 *   - the local normal comes from v = sum c_i (f_i - f_i^eq) + dt_(phi u)/2,
 *     n = -v/|v|, which is the Chapman-Enskog relation of Sec. 3.1 with the
 *     counter term of Eq. 5 substituted;
 *   - the local temperature gradient is -sum c_i (h_i - w_i T)/(tau_h c_s^2),
 *     the first-moment relation of the Chapman-Enskog analysis of Sec. 3.2;
 *   - in the modified thermal LBE both heat capacitances multiply at the
 *     destination node x + c_i and time t; the source term uses the source node;
 *   - isotropic D2Q9 stencils with mirror/Dirichlet ghosts for grad phi,
 *     lap phi and grad T (the paper does not say how they are discretised);
 *   - collision of the NS and thermal LBEs: BGK as printed, or (collision = 1)
 *     the two-relaxation-time variant the paper names as a simple extension
 *     (Sec. 3): populations split into parts even and odd under c_i -> -c_i;
 *     the part carrying the transport coefficient keeps the BGK time (even for
 *     the viscosity of the NS LBE, odd for the conductivity of the thermal LBE),
 *     the other one follows from (tau+ - 1/2)(tau- - 1/2) = trt_magic; each
 *     part of the forcing term gets its own factor 1 - 1/(2 tau);
 *   - interfacial force (force_form = 1): the capillary term of Eq. 11 in the
 *     potential form -phi grad mu_phi (not in the paper; equal to mu_phi grad phi
 *     up to a gradient), mu_phi on the first ghost ring from phi extended to a
 *     second ring by the same ghost rules, grad mu_phi by the isotropic stencil;
 *   - halfway bounce-back walls, anti-bounce-back Dirichlet temperature walls,
 *     bounce-back adiabatic walls; inlet: anti-bounce-back for phi and T and
 *     moving-wall bounce-back for the inflow velocity; outlet: anti-bounce-back
 *     at pressure 0 with the node's own velocity, phi and T.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---- D2Q9 lattice (Sec. 4, preamble): c_0=(0,0); c_1..4 axis; c_5..8 diagonal ---- */
static const int CX[9] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int CY[9] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const double WI[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
static const int OPP[9] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
static const double CS2 = 1.0 / 3.0;

/* boundary kinds per side */
enum { ORC_PERIODIC = 0, ORC_WALL_T = 1, ORC_WALL_ADIABATIC = 2, ORC_INLET = 3, ORC_OUTLET = 4 };
/* sides */
enum { XLO = 0, XHI = 1, YLO = 2, YHI = 3 };

typedef struct {
    int32_t nx, ny;
    int32_t bc[4];      /* x-lo, x-hi, y-lo, y-hi */
    int32_t grad_mode;  /* 0: normal and grad T from moments; 1: from the stencils */
    int32_t n_bubbles;  /* number of tracked light-phase regions (<= 4) */
    int32_t collision;  /* 0: BGK; 1: two-relaxation-time for the NS and thermal LBEs */
    int32_t force_form; /* 0: capillary term (sigma/W^2) mu_phi grad phi, final form of Eq. 11;
                           1: potential form -(sigma/W^2) phi grad mu_phi */
    double trt_magic;   /* (tau+ - 1/2)(tau- - 1/2) of the two-relaxation-time collision */
    double rho_l, rho_h, mu_l, mu_h, lam_l, lam_h, rcp_l, rcp_h;
    double sigma_ref, sigma_T, sigma_TT, T_ref;
    double W, M;
    double Gx, Gy;
    double tw_mean[4], tw_amp[4], tw_k[4], tw_slope[4];
    double u_in, phi_in, T_in;
    double bubble_x[4], bubble_y[4];
} orc_params;

typedef struct {
    int64_t step;
    double mass_phi;   /* sum phi */
    double vol_light;  /* sum (1 - phi)/2 */
    double heat;       /* sum rho c_p T */
    double sum_neg;    /* sum_{phi<0} phi */
    double u_r;        /* sum_{phi<0} phi u_y / sum_{phi<0} phi */
    double ux_r;       /* sum_{phi<0} phi u_x / sum_{phi<0} phi */
    double xc, yc;     /* phi-weighted centroid of the phi<0 region */
    double max_u;
    int64_t n_nonfinite;
    int64_t n_neg;
    double bub_x[4], bub_y[4], bub_ux[4], bub_uy[4], bub_sum[4];
} orc_diag;

typedef struct {
    orc_params p;
    int64_t step;
    size_t n;
    double *f, *g, *h;      /* populations at time t, [9][n] */
    double *f2, *g2, *h2;   /* populations at time t+1 */
    double *jx0, *jy0;      /* (phi u) at time t-1 */
    /* pass-1 macroscopic fields */
    double *phi, *T, *ux, *uy, *pr, *Fx, *Fy;
    double *dphx, *dphy, *lphi, *dTx, *dTy;
    double *jx, *jy;
    double *phipad, *Tpad; /* (nx+2)*(ny+2), ghost ring included */
    double *mupad;         /* mu_phi on the same padded grid (potential form only) */
    double bx[4], by[4];    /* previous bubble centroids */
    int* writes;            /* when non-NULL: writes per slot of the new level, [3][9][n] */
} orc_state;

/* ---- constitutive relations ---- */

/* linear interpolation of a property in the order parameter (Sec. 4, preamble) */
static double interp(double xi_l, double xi_h, double phi)
{
    const double phl = -1.0, phh = 1.0;
    return (phi - phh) / (phl - phh) * xi_l + (phi - phl) / (phh - phl) * xi_h;
}

/* surface tension: linear law of Sec. 2 plus the parabolic term of Eq. 63 */
static double sigma_of(const orc_params* P, double T)
{
    double d = T - P->T_ref;
    return P->sigma_ref + P->sigma_T * d + 0.5 * P->sigma_TT * d * d;
}
static double dsigma_dT(const orc_params* P, double T)
{
    return P->sigma_T + P->sigma_TT * (T - P->T_ref);
}

/* wall temperature T_w(s) = mean + amp cos(k s) + slope s along side `side` */
static double wall_T(const orc_params* P, int side, double s)
{
    return P->tw_mean[side] + P->tw_amp[side] * cos(P->tw_k[side] * s) + P->tw_slope[side] * s;
}

/* inflow velocity at a point of an inlet side: fully developed profile
 * 6 u_ave s'(H - s')/H^2 (Sec. 4.3) along the inward normal, s' = s + 1/2 */
static void inlet_u(const orc_params* P, int side, double s, double* ux, double* uy)
{
    double H = (side == XLO || side == XHI) ? (double)P->ny : (double)P->nx;
    double sp = s + 0.5;
    double un = 6.0 * P->u_in * sp * (H - sp) / (H * H);
    *ux = 0.0;
    *uy = 0.0;
    if (side == XLO) *ux = un;
    if (side == XHI) *ux = -un;
    if (side == YLO) *uy = un;
    if (side == YHI) *uy = -un;
}

/* ---- ghost values for the stencils ---- */

enum { KIND_PHI = 0, KIND_T = 1 };

static double ghost_rule(const orc_params* P, int side, int kind, double inner, double s)
{
    int bc = P->bc[side];
    if (kind == KIND_PHI) {
        if (bc == ORC_INLET) return 2.0 * P->phi_in - inner;
        return inner; /* walls: neutral wetting mirror; outlet: zero gradient */
    }
    if (bc == ORC_WALL_T) return 2.0 * wall_T(P, side, s) - inner;
    if (bc == ORC_INLET) return 2.0 * P->T_in - inner;
    return inner; /* adiabatic wall, outlet */
}

/* scalar field value at lattice point (i, j), which may lie outside the domain */
static double field_at(const orc_state* S, const double* s, int kind, int i, int j)
{
    const orc_params* P = &S->p;
    int nx = P->nx, ny = P->ny;
    if (j < 0 || j >= ny) {
        int side = j < 0 ? YLO : YHI;
        if (P->bc[side] == ORC_PERIODIC) return field_at(S, s, kind, i, (j + ny) % ny);
        int jm = j < 0 ? -1 - j : 2 * ny - 1 - j;
        return ghost_rule(P, side, kind, field_at(S, s, kind, i, jm), (double)i);
    }
    if (i < 0 || i >= nx) {
        int side = i < 0 ? XLO : XHI;
        if (P->bc[side] == ORC_PERIODIC) return field_at(S, s, kind, (i + nx) % nx, j);
        int im = i < 0 ? -1 - i : 2 * nx - 1 - i;
        return ghost_rule(P, side, kind, field_at(S, s, kind, im, j), (double)j);
    }
    return s[(size_t)j * nx + i];
}

/* ---- pass 1: macroscopic fields (Sec. 3.1, Sec. 3.2, Sec. 4 preamble) ---- */

static void macros(orc_state* S)
{
    const orc_params* P = &S->p;
    const int nx = P->nx, ny = P->ny;
    const size_t n = S->n;

    /* zeroth moments: phi = sum f_i, T = sum h_i */
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t x = (size_t)j * nx + i;
            double sf = 0.0, sh = 0.0;
            for (int k = 0; k < 9; ++k) {
                sf += S->f[k * n + x];
                sh += S->h[k * n + x];
            }
            S->phi[x] = sf;
            S->T[x] = sh;
        }

    /* phi and T on a padded grid: interior copies plus the ghost ring */
    const int px = nx + 2;
#pragma omp parallel for schedule(static)
    for (int j = -1; j <= ny; ++j)
        for (int i = -1; i <= nx; ++i) {
            size_t q = (size_t)(j + 1) * px + (i + 1);
            S->phipad[q] = field_at(S, S->phi, KIND_PHI, i, j);
            S->Tpad[q] = field_at(S, S->T, KIND_T, i, j);
        }

    /* potential form: mu_phi on the padded grid.  A ghost node takes the
     * formula of Sec. 2 applied to the ghost values of phi, which extend to
     * two nodes beyond the lattice by the same rules as the first ring. */
    if (P->force_form == 1) {
#pragma omp parallel for schedule(static)
        for (int j = -1; j <= ny; ++j)
            for (int i = -1; i <= nx; ++i) {
                double pc = field_at(S, S->phi, KIND_PHI, i, j);
                double lap = 0.0;
                for (int k = 1; k < 9; ++k)
                    lap += 2.0 * WI[k] * (field_at(S, S->phi, KIND_PHI, i + CX[k], j + CY[k]) - pc) / CS2;
                const double phl = -1.0, phh = 1.0;
                S->mupad[(size_t)(j + 1) * px + (i + 1)] =
                    (pc - phl) * (pc - phh) * (pc - 0.5 * (phl + phh)) - P->W * P->W * lap;
            }
    }

#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t x = (size_t)j * nx + i;
            double phi = S->phi[x], T = S->T[x];

            /* isotropic stencils: grad psi = (1/c_s^2) sum w_i c_i psi(x+c_i),
             * lap psi = (2/c_s^2) sum_{i>0} w_i (psi(x+c_i) - psi(x)) */
            double gpx = 0.0, gpy = 0.0, lap = 0.0, gtx = 0.0, gty = 0.0;
            for (int k = 0; k < 9; ++k) {
                size_t q = (size_t)(j + 1 + CY[k]) * px + (i + 1 + CX[k]);
                double pn = S->phipad[q];
                double tn = S->Tpad[q];
                gpx += WI[k] * CX[k] * pn / CS2;
                gpy += WI[k] * CY[k] * pn / CS2;
                gtx += WI[k] * CX[k] * tn / CS2;
                gty += WI[k] * CY[k] * tn / CS2;
                if (k > 0) lap += 2.0 * WI[k] * (pn - phi) / CS2;
            }
            S->dphx[x] = gpx;
            S->dphy[x] = gpy;
            S->lphi[x] = lap;
            S->dTx[x] = gtx;
            S->dTy[x] = gty;

            /* density (Eq. 8) and its gradient */
            double rho = interp(P->rho_l, P->rho_h, phi);
            double drho = (P->rho_l - P->rho_h) / (-1.0 - 1.0);
            double grx = drho * gpx, gry = drho * gpy;

            /* chemical potential: double-well bulk term minus W^2 lap phi (Sec. 2) */
            const double phl = -1.0, phh = 1.0;
            double mu_phi = (phi - phl) * (phi - phh) * (phi - 0.5 * (phl + phh)) - P->W * P->W * lap;

            /* surface tension and its gradient through T */
            double sig = sigma_of(P, T);
            double dsig = dsigma_dT(P, T);
            double gsx = dsig * gtx, gsy = dsig * gty;

            /* interfacial force, final form of Eq. 11; the potential form
             * replaces its capillary term mu_phi grad phi by -phi grad mu_phi
             * (the two differ by the gradient of phi mu_phi) */
            double g2 = gpx * gpx + gpy * gpy;
            double sdotp = gsx * gpx + gsy * gpy;
            double pref = 3.0 * sqrt(2.0) * P->W / 4.0;
            double capx = mu_phi * gpx, capy = mu_phi * gpy;
            if (P->force_form == 1) {
                double gmx = 0.0, gmy = 0.0;
                for (int k = 0; k < 9; ++k) {
                    double mn = S->mupad[(size_t)(j + 1 + CY[k]) * px + (i + 1 + CX[k])];
                    gmx += WI[k] * CX[k] * mn / CS2;
                    gmy += WI[k] * CY[k] * mn / CS2;
                }
                capx = -phi * gmx;
                capy = -phi * gmy;
            }
            double Fx = pref * (g2 * gsx - sdotp * gpx + sig / (P->W * P->W) * capx) + P->Gx;
            double Fy = pref * (g2 * gsy - sdotp * gpy + sig / (P->W * P->W) * capy) + P->Gy;
            S->Fx[x] = Fx;
            S->Fy[x] = Fy;

            /* momentum: rho u = sum c_i g_i + F/2 (Sec. 3.1) */
            double mx = 0.0, my = 0.0, sg = 0.0;
            for (int k = 0; k < 9; ++k) {
                double gk = S->g[k * n + x];
                mx += CX[k] * gk;
                my += CY[k] * gk;
                if (k > 0) sg += gk;
            }
            double ux = (mx + 0.5 * Fx) / rho;
            double uy = (my + 0.5 * Fy) / rho;
            S->ux[x] = ux;
            S->uy[x] = uy;

            /* pressure: c_s^2/(1-w_0) [sum_{i>0} g_i + u.grad rho/2 + rho s_0(u)] */
            double uu = ux * ux + uy * uy;
            double s0 = WI[0] * (-uu / (2.0 * CS2));
            S->pr[x] = CS2 / (1.0 - WI[0]) * (sg + 0.5 * (ux * grx + uy * gry) + rho * s0);

            S->jx[x] = phi * ux;
            S->jy[x] = phi * uy;
        }
}

/* ---- pass 2: collisions (Eq. 14, the NS LBE, Eq. 28) and push streaming ---- */

/* stores into the new time level; counts the stores when checking coverage */
static void put3(orc_state* S, int k, size_t y, double fv, double gv, double hv)
{
    S->f2[k * S->n + y] = fv;
    S->g2[k * S->n + y] = gv;
    S->h2[k * S->n + y] = hv;
    if (S->writes) {
#pragma omp atomic
        S->writes[k * S->n + y] += 1;
    }
}

static void collide_stream(orc_state* S)
{
    const orc_params* P = &S->p;
    const int nx = P->nx, ny = P->ny;
    const size_t n = S->n;
    const double tau_phi = 0.5 + P->M / CS2; /* M = c_s^2 (tau_phi - 1/2) */

#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t x = (size_t)j * nx + i;
            double phi = S->phi[x], T = S->T[x];
            double ux = S->ux[x], uy = S->uy[x], pr = S->pr[x];
            double Fx = S->Fx[x], Fy = S->Fy[x];
            double rho = interp(P->rho_l, P->rho_h, phi);
            double mu = interp(P->mu_l, P->mu_h, phi);
            double lam = interp(P->lam_l, P->lam_h, phi);
            double rcp = interp(P->rcp_l, P->rcp_h, phi);
            double tau_g = 0.5 + mu / (rho * CS2);  /* mu = rho c_s^2 (tau_g - 1/2) */
            double tau_h = 0.5 + lam / CS2;          /* lambda = c_s^2 (tau_h - 1/2) */
            double drho = (P->rho_l - P->rho_h) / (-1.0 - 1.0);
            double grx = drho * S->dphx[x], gry = drho * S->dphy[x];

            /* time derivative of phi u by the first-order Euler scheme (Sec. 4) */
            double djx = S->jx[x] - S->jx0[x];
            double djy = S->jy[x] - S->jy0[x];

            double fk[9], gk[9], hk[9];
            for (int k = 0; k < 9; ++k) {
                fk[k] = S->f[k * n + x];
                gk[k] = S->g[k * n + x];
                hk[k] = S->h[k * n + x];
            }

            /* AC LBE: equilibrium and local unit normal */
            double feq[9];
            for (int k = 0; k < 9; ++k) feq[k] = WI[k] * phi * (1.0 + (CX[k] * ux + CY[k] * uy) / CS2);
            double nxv = 0.0, nyv = 0.0;
            if (P->grad_mode == 0) {
                double vx = 0.0, vy = 0.0;
                for (int k = 0; k < 9; ++k) {
                    vx += CX[k] * (fk[k] - feq[k]);
                    vy += CY[k] * (fk[k] - feq[k]);
                }
                vx += 0.5 * djx;
                vy += 0.5 * djy;
                double vn = sqrt(vx * vx + vy * vy);
                if (vn > 1e-300) {
                    nxv = -vx / vn;
                    nyv = -vy / vn;
                }
            } else {
                double gx = S->dphx[x], gy = S->dphy[x];
                double gn = sqrt(gx * gx + gy * gy);
                if (gn > 1e-300) {
                    nxv = gx / gn;
                    nyv = gy / gn;
                }
            }
            double lamc = (1.0 - phi * phi) / (sqrt(2.0) * P->W);

            /* NS LBE force term needs u.grad rho */
            double ugr = ux * grx + uy * gry;
            double uu = ux * ux + uy * uy;

            /* thermal LBE: local grad T and source */
            double tgx, tgy;
            if (P->grad_mode == 0) {
                double mx = 0.0, my = 0.0;
                for (int k = 0; k < 9; ++k) {
                    mx += CX[k] * (hk[k] - WI[k] * T);
                    my += CY[k] * (hk[k] - WI[k] * T);
                }
                tgx = -mx / (tau_h * CS2);
                tgy = -my / (tau_h * CS2);
            } else {
                tgx = S->dTx[x];
                tgy = S->dTy[x];
            }
            double Fhat = -rcp * (ux * tgx + uy * tgy);

            double fs[9], gs[9], hs[9], geq[9], Gi[9];
            for (int k = 0; k < 9; ++k) {
                double cu = CX[k] * ux + CY[k] * uy;
                /* Eq. 14 with source R_i */
                double Ri = WI[k] * (CX[k] * (djx + CS2 * nxv * lamc) + CY[k] * (djy + CS2 * nyv * lamc)) / CS2;
                fs[k] = fk[k] - (fk[k] - feq[k]) / tau_phi + (1.0 - 1.0 / (2.0 * tau_phi)) * Ri;

                /* NS LBE: equilibrium with s_i(u) and forcing G_i */
                double si = WI[k] * (cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
                geq[k] = (k == 0 ? pr / CS2 * (WI[0] - 1.0) : pr / CS2 * WI[k]) + rho * si;
                /* u grad rho : (c_i c_i - c_s^2 I) */
                double tens = ux * grx * (CX[k] * CX[k] - CS2) + ux * gry * (CX[k] * CY[k])
                            + uy * grx * (CY[k] * CX[k]) + uy * gry * (CY[k] * CY[k] - CS2);
                Gi[k] = WI[k] * (ugr + (CX[k] * Fx + CY[k] * Fy) / CS2 + tens / CS2);
            }
            if (P->collision == 0) {
                for (int k = 0; k < 9; ++k) {
                    gs[k] = gk[k] - (gk[k] - geq[k]) / tau_g + (1.0 - 1.0 / (2.0 * tau_g)) * Gi[k];
                    /* Eq. 28 collision part: h_i - (h_i - h_i^eq)/tau_h + Fhat_i */
                    hs[k] = hk[k] - (hk[k] - WI[k] * T) / tau_h + WI[k] * Fhat;
                }
            } else {
                /* two relaxation times: even part (+) and odd part (-) of each
                   population, equilibrium and forcing term */
                double tgp = tau_g, tgm = 0.5 + P->trt_magic / (tau_g - 0.5);
                double thm = tau_h, thp = 0.5 + P->trt_magic / (tau_h - 0.5);
                for (int k = 0; k < 9; ++k) {
                    int kb = OPP[k];
                    double gp = 0.5 * (gk[k] + gk[kb]), gm = 0.5 * (gk[k] - gk[kb]);
                    double ep = 0.5 * (geq[k] + geq[kb]), em = 0.5 * (geq[k] - geq[kb]);
                    double Gp = 0.5 * (Gi[k] + Gi[kb]), Gm = 0.5 * (Gi[k] - Gi[kb]);
                    gs[k] = gk[k] - (gp - ep) / tgp - (gm - em) / tgm
                          + (1.0 - 1.0 / (2.0 * tgp)) * Gp + (1.0 - 1.0 / (2.0 * tgm)) * Gm;
                    double hp = 0.5 * (hk[k] + hk[kb]), hm = 0.5 * (hk[k] - hk[kb]);
                    /* h_i^eq = w_i T and the source w_i Fhat are even */
                    hs[k] = hk[k] - (hp - WI[k] * T) / thp - hm / thm + WI[k] * Fhat;
                }
            }
            (void)rcp;

            /* streaming */
            for (int k = 0; k < 9; ++k) {
                int ti = i + CX[k], tj = j + CY[k];
                int outx = 0, outy = 0;
                if (ti < 0 || ti >= nx) {
                    if (P->bc[ti < 0 ? XLO : XHI] == ORC_PERIODIC) ti = (ti + nx) % nx;
                    else outx = 1;
                }
                if (tj < 0 || tj >= ny) {
                    if (P->bc[tj < 0 ? YLO : YHI] == ORC_PERIODIC) tj = (tj + ny) % ny;
                    else outy = 1;
                }
                if (!outx && !outy) {
                    size_t y = (size_t)tj * nx + ti;
                    double rcpy = interp(P->rcp_l, P->rcp_h, S->phi[y]);
                    /* Eq. 28: rcp(y) h_i(y,t+1) = h*_i(x) + (rcp(y) - 1) h_i(y,t) */
                    put3(S, k, y, fs[k], gs[k], (hs[k] + (rcpy - 1.0) * S->h[k * n + y]) / rcpy);
                    continue;
                }
                /* which side's rule applies: walls before the inlet before the outlet */
                int sx = i + CX[k] < 0 ? XLO : XHI;
                int sy = j + CY[k] < 0 ? YLO : YHI;
                int side;
                if (outx && outy) {
                    int bx = P->bc[sx], by = P->bc[sy];
                    int px = (bx == ORC_WALL_T || bx == ORC_WALL_ADIABATIC) ? 2 : (bx == ORC_INLET ? 1 : 0);
                    int py = (by == ORC_WALL_T || by == ORC_WALL_ADIABATIC) ? 2 : (by == ORC_INLET ? 1 : 0);
                    side = px > py ? sx : sy;
                } else {
                    side = outx ? sx : sy;
                }
                /* coordinate of the wall crossing point along the side */
                double s = (side == XLO || side == XHI) ? j + 0.5 * CY[k] : i + 0.5 * CX[k];
                int kb = OPP[k];
                int bc = P->bc[side];
                double fb, gb, hb;
                if (bc == ORC_WALL_T || bc == ORC_WALL_ADIABATIC) {
                    /* halfway bounce-back */
                    fb = fs[k];
                    gb = gs[k];
                    if (bc == ORC_WALL_T) hb = -hs[k] + 2.0 * WI[k] * wall_T(P, side, s);
                    else hb = hs[k];
                } else if (bc == ORC_INLET) {
                    /* anti-bounce-back for phi and T, moving-wall bounce-back for u */
                    double uix, uiy;
                    inlet_u(P, side, s, &uix, &uiy);
                    fb = -fs[k] + 2.0 * WI[k] * P->phi_in;
                    gb = gs[k] - 2.0 * WI[k] * rho * (CX[k] * uix + CY[k] * uiy) / CS2;
                    hb = -hs[k] + 2.0 * WI[k] * P->T_in;
                } else {
                    /* outlet: anti-bounce-back at pressure 0 with the node's own
                     * velocity, phi and T (open, zero normal gradient) */
                    double cu = CX[k] * ux + CY[k] * uy;
                    double uu = ux * ux + uy * uy;
                    fb = -fs[k] + 2.0 * WI[k] * phi;
                    gb = -gs[k] + 2.0 * WI[k] * rho * (cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
                    hb = -hs[k] + 2.0 * WI[k] * T;
                }
                put3(S, kb, x, fb, gb, (hb + (rcp - 1.0) * S->h[kb * n + x]) / rcp);
            }
        }
}

/* ---- public API ---- */

#define API __attribute__((visibility("default")))

static void* xcalloc(size_t count)
{
    return calloc(count, sizeof(double));
}

API void orc_destroy(orc_state* S)
{
    if (!S) return;
    double** bufs[] = {&S->f, &S->g, &S->h, &S->f2, &S->g2, &S->h2, &S->jx0, &S->jy0,
                       &S->phi, &S->T, &S->ux, &S->uy, &S->pr, &S->Fx, &S->Fy,
                       &S->dphx, &S->dphy, &S->lphi, &S->dTx, &S->dTy, &S->jx, &S->jy, &S->phipad, &S->Tpad,
                       &S->mupad};
    for (size_t b = 0; b < sizeof(bufs) / sizeof(bufs[0]); ++b) free(*bufs[b]);
    free(S->writes);
    free(S);
}

/* Creates a state with populations at equilibrium for the given initial fields
 * (p = 0), then sets (phi u)_{t-1} = (phi u)_t so that the first time derivative
 * of phi u is zero.  Fields are host arrays of nx*ny doubles, x fastest.
 * Returns NULL on invalid parameters or allocation failure. */
API orc_state* orc_create(const orc_params* P, const double* phi0, const double* ux0,
                          const double* uy0, const double* T0)
{
    if (!P || P->nx < 3 || P->ny < 3 || P->n_bubbles < 0 || P->n_bubbles > 4) return NULL;
    if (P->force_form != 0 && P->force_form != 1) return NULL;
    if ((P->bc[XLO] == ORC_PERIODIC) != (P->bc[XHI] == ORC_PERIODIC)) return NULL;
    if ((P->bc[YLO] == ORC_PERIODIC) != (P->bc[YHI] == ORC_PERIODIC)) return NULL;
    orc_state* S = (orc_state*)calloc(1, sizeof(orc_state));
    if (!S) return NULL;
    S->p = *P;
    S->n = (size_t)P->nx * P->ny;
    size_t n = S->n;
    S->f = xcalloc(9 * n); S->g = xcalloc(9 * n); S->h = xcalloc(9 * n);
    S->f2 = xcalloc(9 * n); S->g2 = xcalloc(9 * n); S->h2 = xcalloc(9 * n);
    S->jx0 = xcalloc(n); S->jy0 = xcalloc(n);
    S->phi = xcalloc(n); S->T = xcalloc(n); S->ux = xcalloc(n); S->uy = xcalloc(n);
    S->pr = xcalloc(n); S->Fx = xcalloc(n); S->Fy = xcalloc(n);
    S->dphx = xcalloc(n); S->dphy = xcalloc(n); S->lphi = xcalloc(n);
    S->dTx = xcalloc(n); S->dTy = xcalloc(n); S->jx = xcalloc(n); S->jy = xcalloc(n);
    S->phipad = xcalloc((size_t)(P->nx + 2) * (P->ny + 2));
    S->Tpad = xcalloc((size_t)(P->nx + 2) * (P->ny + 2));
    S->mupad = xcalloc((size_t)(P->nx + 2) * (P->ny + 2));
    if (!S->f || !S->g || !S->h || !S->f2 || !S->g2 || !S->h2 || !S->jx0 || !S->jy0 || !S->phi ||
        !S->T || !S->ux || !S->uy || !S->pr || !S->Fx || !S->Fy || !S->dphx || !S->dphy ||
        !S->lphi || !S->dTx || !S->dTy || !S->jx || !S->jy || !S->phipad || !S->Tpad ||
        !S->mupad) {
        orc_destroy(S);
        return NULL;
    }
    for (size_t x = 0; x < n; ++x) {
        double phi = phi0[x], ux = ux0[x], uy = uy0[x], T = T0[x];
        double rho = interp(P->rho_l, P->rho_h, phi);
        double uu = ux * ux + uy * uy;
        for (int k = 0; k < 9; ++k) {
            double cu = CX[k] * ux + CY[k] * uy;
            S->f[k * n + x] = WI[k] * phi * (1.0 + cu / CS2);
            S->g[k * n + x] = rho * WI[k] * (cu / CS2 + cu * cu / (2.0 * CS2 * CS2) - uu / (2.0 * CS2));
            S->h[k * n + x] = WI[k] * T;
        }
    }
    macros(S);
    memcpy(S->jx0, S->jx, n * sizeof(double));
    memcpy(S->jy0, S->jy, n * sizeof(double));
    for (int b = 0; b < 4; ++b) {
        S->bx[b] = P->bubble_x[b];
        S->by[b] = P->bubble_y[b];
    }
    return S;
}

/* Advances the state by n time steps. */
API void orc_step(orc_state* S, int64_t nsteps)
{
    for (int64_t s = 0; s < nsteps; ++s) {
        macros(S);
        collide_stream(S);
        double* t;
        t = S->f; S->f = S->f2; S->f2 = t;
        t = S->g; S->g = S->g2; S->g2 = t;
        t = S->h; S->h = S->h2; S->h2 = t;
        memcpy(S->jx0, S->jx, S->n * sizeof(double));
        memcpy(S->jy0, S->jy, S->n * sizeof(double));
        S->step++;
    }
}

/* Macroscopic fields at the current time (any output pointer may be NULL). */
API void orc_fields(orc_state* S, double* phi, double* ux, double* uy, double* T, double* p)
{
    macros(S);
    size_t b = S->n * sizeof(double);
    if (phi) memcpy(phi, S->phi, b);
    if (ux) memcpy(ux, S->ux, b);
    if (uy) memcpy(uy, S->uy, b);
    if (T) memcpy(T, S->T, b);
    if (p) memcpy(p, S->pr, b);
}

/* Every pass-1 quantity, for unit tests: 13 planes of nx*ny doubles in the order
 * phi, T, ux, uy, p, Fx, Fy, dphi/dx, dphi/dy, lap phi, dT/dx, dT/dy, phi*u_y. */
API void orc_macros_all(orc_state* S, double* out)
{
    macros(S);
    const double* src[13] = {S->phi, S->T, S->ux, S->uy, S->pr, S->Fx, S->Fy,
                             S->dphx, S->dphy, S->lphi, S->dTx, S->dTy, S->jy};
    for (int q = 0; q < 13; ++q) memcpy(out + q * S->n, src[q], S->n * sizeof(double));
}

/* Copies populations out: f, g, h each [9][nx*ny]; j_prev [2][nx*ny]. */
API void orc_get_state(const orc_state* S, double* f, double* g, double* h, double* jprev, int64_t* step)
{
    size_t b = 9 * S->n * sizeof(double);
    if (f) memcpy(f, S->f, b);
    if (g) memcpy(g, S->g, b);
    if (h) memcpy(h, S->h, b);
    if (jprev) {
        memcpy(jprev, S->jx0, S->n * sizeof(double));
        memcpy(jprev + S->n, S->jy0, S->n * sizeof(double));
    }
    if (step) *step = S->step;
}

/* Replaces populations (any pointer may be NULL to keep the current one). */
API void orc_set_state(orc_state* S, const double* f, const double* g, const double* h,
                       const double* jprev, int64_t step)
{
    size_t b = 9 * S->n * sizeof(double);
    if (f) memcpy(S->f, f, b);
    if (g) memcpy(S->g, g, b);
    if (h) memcpy(S->h, h, b);
    if (jprev) {
        memcpy(S->jx0, jprev, S->n * sizeof(double));
        memcpy(S->jy0, jprev + S->n, S->n * sizeof(double));
    }
    S->step = step;
}

/* Diagnostics: global sums, the droplet velocity of Sec. 4.2 and the per-bubble
 * velocity and position of Sec. 4.3 (light-phase nodes assigned to the nearest
 * previous centroid, ties to the lower index). */
API void orc_diagnostics(orc_state* S, orc_diag* D)
{
    const orc_params* P = &S->p;
    macros(S);
    memset(D, 0, sizeof(*D));
    D->step = S->step;
    double sx = 0.0, sy = 0.0, sux = 0.0, suy = 0.0;
    double bs[4] = {0}, bxs[4] = {0}, bys[4] = {0}, bux[4] = {0}, buy[4] = {0};
    for (int j = 0; j < P->ny; ++j)
        for (int i = 0; i < P->nx; ++i) {
            size_t x = (size_t)j * P->nx + i;
            double phi = S->phi[x], T = S->T[x], ux = S->ux[x], uy = S->uy[x];
            if (!isfinite(phi) || !isfinite(T) || !isfinite(ux) || !isfinite(uy) || !isfinite(S->pr[x])) {
                D->n_nonfinite++;
                continue;
            }
            D->mass_phi += phi;
            D->vol_light += 0.5 * (1.0 - phi);
            D->heat += interp(P->rcp_l, P->rcp_h, phi) * T;
            double um = sqrt(ux * ux + uy * uy);
            if (um > D->max_u) D->max_u = um;
            if (phi < 0.0) {
                D->n_neg++;
                D->sum_neg += phi;
                sux += phi * ux;
                suy += phi * uy;
                sx += phi * i;
                sy += phi * j;
                if (P->n_bubbles > 0) {
                    int best = 0;
                    double bd = 0.0;
                    for (int b = 0; b < P->n_bubbles; ++b) {
                        double dx = i - S->bx[b], dy = j - S->by[b];
                        double d2 = dx * dx + dy * dy;
                        if (b == 0 || d2 < bd) {
                            bd = d2;
                            best = b;
                        }
                    }
                    bs[best] += phi;
                    bxs[best] += phi * i;
                    bys[best] += phi * j;
                    bux[best] += phi * ux;
                    buy[best] += phi * uy;
                }
            }
        }
    if (D->sum_neg != 0.0) {
        D->u_r = suy / D->sum_neg;
        D->ux_r = sux / D->sum_neg;
        D->xc = sx / D->sum_neg;
        D->yc = sy / D->sum_neg;
    }
    for (int b = 0; b < P->n_bubbles; ++b) {
        D->bub_sum[b] = bs[b];
        if (bs[b] != 0.0) {
            D->bub_x[b] = bxs[b] / bs[b];
            D->bub_y[b] = bys[b] / bs[b];
            D->bub_ux[b] = bux[b] / bs[b];
            D->bub_uy[b] = buy[b] / bs[b];
            S->bx[b] = D->bub_x[b];
            S->by[b] = D->bub_y[b];
        } else {
            D->bub_x[b] = S->bx[b];
            D->bub_y[b] = S->by[b];
        }
    }
}

/* One step that also counts the stores into every slot of the new time level;
 * counts[9][n] receives them (each must be exactly 1). */
API int orc_step_count_writes(orc_state* S, int* counts)
{
    S->writes = (int*)calloc(9 * S->n, sizeof(int));
    if (!S->writes) return -1;
    orc_step(S, 1);
    memcpy(counts, S->writes, 9 * S->n * sizeof(int));
    free(S->writes);
    S->writes = NULL;
    return 0;
}

API void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

API int orc_get_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

API int orc_sizeof_params(void) { return (int)sizeof(orc_params); }
API int orc_sizeof_diag(void) { return (int)sizeof(orc_diag); }
