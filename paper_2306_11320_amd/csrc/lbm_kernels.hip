// gfx950 kernels for one time step of the three coupled D2Q9 lattice Boltzmann
// equations of Wang, He & Wang, arXiv:2306.11320 (Sec. 3, Sec. 4 preamble).
//
// One fused kernel per step.  A workgroup owns a TX x TY tile of nodes, one
// work-item per node:
//   1. every work-item loads its own 27 populations and (phi u) of the previous
//      level; the zeroth moments phi = sum f_i, T = sum h_i and the h_i of the
//      tile plus a one-node ring go to LDS (the ring re-sums its neighbours'
//      populations, which mostly hit L2);
//   2. isotropic stencils for grad phi, lap phi, grad T from LDS; properties,
//      sigma(T), the interfacial force of Eq. 11, u and p (Sec. 3.1), the time
//      derivative of phi u (Sec. 4 preamble);
//   3. the three collisions (Eq. 14, the NS LBE, Eq. 28): BGK, or two
//      relaxation times for the NS and thermal LBEs (a separate kernel, used
//      when some lattice of the launch asks for it);
//   4. push streaming to the other time level with the boundary rules folded
//      in; the thermal update divides by the destination's heat capacitance
//      and blends with the destination's old h_i, both read from LDS.
// There is no MFMA on this path: it is bound by HBM traffic.
//
// Storage: nodes x fastest in blocks of 64 consecutive nodes of a row, each
// block holding the 27 populations as runs of 64 values; f and h kept as
// deviations from w_i phi0 and w_i T0 (exact for BGK, streaming, bounce-back
// and the blend, whose weights sum to one), g as is.  The base of each
// population of each time level comes precomputed in the lattice's parameter
// block.
#include "lbm_internal.hpp"

#include <type_traits>

namespace lbm {

// Global-memory views of the lattice pointers: accesses through them compile
// to global_* instructions; generic pointers give flat_* ones, which also
// count against the LDS wait counter and so stall behind the patch traffic.
template <typename T>
using gptr = __attribute__((address_space(1))) T*;
template <typename T>
__device__ inline gptr<T> to_global(T* p) { return (gptr<T>)p; }

// Reciprocals: the hardware's (1 ulp) in FP32, correctly rounded in FP64.
// The FP32 reciprocal square root flushes subnormal inputs, so unit vectors
// are only formed from squared lengths of at least the smallest normal
// float (below it the direction is rounding noise and the vector is zero).
__device__ inline float recip(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ inline double recip(double x) { return 1.0 / x; }
__device__ inline float rsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ inline double rsq(double x) { return 1.0 / sqrt(x); }
__device__ inline bool has_direction(float n2) { return n2 >= 1.17549435e-38f; }
__device__ inline bool has_direction(double n2) { return n2 > 0.0; }

// Node offsets within a time level are 32-bit byte offsets (the host keeps a
// level below 4 GiB); the population base is uniform, so loads and stores take
// a scalar base and a 32-bit vector offset.
// Base of population q of time level `lev`, read from the lattice's parameter
// block (a scalar load).
template <typename real>
__device__ inline gptr<const real> src_plane(const Inst<real>& I, int lev, int q)
{
    return to_global<const real>(I.qbase[lev][q]);
}
template <typename real>
__device__ inline gptr<real> dst_plane(const Inst<real>& I, int lev, int q)
{
    return to_global(I.qbase[lev][q]);
}
// Byte offset of node idx from the base of any population of its level: the
// populations of kBlock consecutive nodes (one row segment) are stored as 27
// runs of kBlock values, block after block.
template <typename real>
__device__ inline unsigned noff(unsigned idx)
{
    return ((idx / kBlock) * (unsigned)(kPlanes * kBlock) + (idx % kBlock)) * (unsigned)sizeof(real);
}

// Element at a 32-bit byte offset from a (uniform) base.
template <typename T>
__device__ inline T ld(gptr<const T> base, unsigned off) { return *(gptr<const T>)((gptr<const char>)base + off); }
template <typename T>
__device__ inline T ld(gptr<T> base, unsigned off) { return *(gptr<const T>)((gptr<const char>)base + off); }
template <typename T>
__device__ inline void st(gptr<T> base, unsigned off, T v) { *(gptr<T>)((gptr<char>)base + off) = v; }

enum { BC_PERIODIC = 0, BC_WALL_T = 1, BC_WALL_ADIABATIC = 2, BC_INLET = 3, BC_OUTLET = 4 };

// D2Q9 (Sec. 4 preamble): c_0 = (0,0); c_1..4 = (1,0),(0,1),(-1,0),(0,-1);
// c_5..8 = (1,1),(-1,1),(-1,-1),(1,-1); weights 4/9, 1/9, 1/36.
__host__ __device__ constexpr int cx(int k) { return (k == 1 || k == 5 || k == 8) ? 1 : ((k == 3 || k == 6 || k == 7) ? -1 : 0); }
__host__ __device__ constexpr int cy(int k) { return (k == 2 || k == 5 || k == 6) ? 1 : ((k == 4 || k == 7 || k == 8) ? -1 : 0); }
__host__ __device__ constexpr int opp(int k) { return k == 0 ? 0 : (k <= 4 ? ((k + 1) % 4) + 1 : ((k - 3) % 4) + 5); }
template <typename real>
__device__ constexpr real wgt(int k) { return k == 0 ? real(4.0 / 9.0) : (k <= 4 ? real(1.0 / 9.0) : real(1.0 / 36.0)); }

static_assert(opp(1) == 3 && opp(2) == 4 && opp(3) == 1 && opp(4) == 2, "opposite map");
static_assert(opp(5) == 7 && opp(6) == 8 && opp(7) == 5 && opp(8) == 6, "opposite map");

template <typename real, int TX, int TY>
struct Patch {
    static constexpr int PX = TX + 2, PY = TY + 2, NP = PX * PY;
    static constexpr int NRING = 2 * PX + 2 * TY;
    real phi[NP];    // phi - phi0 on the tile plus ring (ghosts applied)
    real T[NP];      // T - T0
    real irc[NP];    // 1 / (rho c_p)
    real h[9][NP];   // h_i - w_i T0 of the node (real nodes only)
};

// Extra LDS of the potential form of the capillary force: phi - phi0 on the
// tile and two rings, and mu_phi on the tile and one ring (the layout of the
// patch's arrays).
template <typename real, int TX, int TY>
struct PotLDS {
    static constexpr int QX = TX + 4, QY = TY + 4;
    real phw[QX * QY];
    real mu[(TX + 2) * (TY + 2)];
};
struct NoPot {};

// Wall temperature relative to T0 at coordinate s = s2 / 2 along `side` (s2 an
// integer: nodes and the half-way points between them), from the table the
// host fills at init with T_w(s) = Tw_mean + Tw_amp cos(Tw_k s) + Tw_slope s.
// An inline FP64 cosine held ~50 VGPRs in the boundary code of the step kernel
// (a wave per SIMD).  Points beyond the table (ghosts of patch entries that no
// stencil reads, in tiles cut by the lattice's end) take its end values.
template <typename real>
__device__ inline real wall_T(const Inst<real>& I, int side, int s2)
{
    const int j = min(max(s2 + kTwPad, 0), I.tw_stride - 1);
    return to_global<const real>(I.twall)[side * I.tw_stride + j];
}

// Affine ghost rule of one side: ghost = a + sgn * inner (deviation units).
template <typename real>
__device__ inline void ghost_rule(const Inst<real>& I, int side, int s2, real& aphi, real& sphi, real& aT, real& sT)
{
    const int bc = I.bc[side];
    aphi = real(0); sphi = real(1); aT = real(0); sT = real(1);
    if (bc == BC_INLET) {
        aphi = real(2) * I.phi_in_d; sphi = real(-1);
        aT = real(2) * I.T_in_d; sT = real(-1);
    } else if (bc == BC_WALL_T) {
        aT = real(2) * wall_T(I, side, s2); sT = real(-1);
    }
}

// Maps lattice point (gx, gy), possibly outside the domain, to the node whose
// moments define it and the affine map applied to them.  The rule of the y
// side is applied outermost, as for the corner ghosts of the oracle's reading.
template <typename real>
__device__ inline bool resolve(const Inst<real>& I, int gx, int gy, int& sx, int& sy, real& aphi, real& sphi,
                               real& aT, real& sT)
{
    const int nx = I.nx, ny = I.ny;
    bool real_node = true;
    real ayp = 0, syp = 1, ayT = 0, syT = 1, axp = 0, sxp = 1, axT = 0, sxT = 1;
    int jj = gy;
    if (gy < 0 || gy >= ny) {
        const int side = gy < 0 ? 2 : 3;
        if (I.bc[side] == BC_PERIODIC) {
            jj = gy < 0 ? gy + ny : gy - ny;
        } else {
            jj = gy < 0 ? -1 - gy : 2 * ny - 1 - gy;
            ghost_rule(I, side, 2 * gx, ayp, syp, ayT, syT);
            real_node = false;
        }
    }
    int ii = gx;
    if (gx < 0 || gx >= nx) {
        const int side = gx < 0 ? 0 : 1;
        if (I.bc[side] == BC_PERIODIC) {
            ii = gx < 0 ? gx + nx : gx - nx;
        } else {
            ii = gx < 0 ? -1 - gx : 2 * nx - 1 - gx;
            ghost_rule(I, side, 2 * jj, axp, sxp, axT, sxT);
            real_node = false;
        }
    }
    // points beyond the one-node ring of the lattice are never read by a
    // stencil; clamping keeps their loads in bounds for tiny lattices
    sx = ii < 0 ? 0 : (ii >= nx ? nx - 1 : ii);
    sy = jj < 0 ? 0 : (jj >= ny ? ny - 1 : jj);
    aphi = ayp + syp * axp;
    sphi = syp * sxp;
    aT = ayT + syT * axT;
    sT = syT * sxT;
    return real_node;
}

// Fills one patch entry from global memory (ring entries and tile entries whose
// node lies outside the lattice).
// Periodic image of a coordinate at most one period outside [0, n).
__device__ inline int wrap1(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

template <typename real, bool EDGE, typename P>
__device__ inline void fill_entry(const Inst<real>& I, int src, P& S, int q, int gx, int gy)
{
    int sx, sy;
    real aphi = 0, sphi = 1, aT = 0, sT = 1;
    bool rn = true;
    if (EDGE) {
        rn = resolve(I, gx, gy, sx, sy, aphi, sphi, aT, sT);
    } else {
        // tile and ring touch no wall, inlet or outlet: at most a periodic wrap
        sx = wrap1(gx, I.nx);
        sy = wrap1(gy, I.ny);
    }
    const unsigned idx = (unsigned)(sy * I.pitch + sx);
    real sf = 0, sh = 0, hk[9];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        sf += ld(src_plane(I, src, kF + k), noff<real>(idx));
        hk[k] = ld(src_plane(I, src, kH + k), noff<real>(idx));
        sh += hk[k];
    }
    const real dphi = (EDGE && !rn) ? aphi + sphi * sf : sf;
    S.phi[q] = dphi;
    S.T[q] = (EDGE && !rn) ? aT + sT * sh : sh;
    S.irc[q] = recip(I.rcp_a + I.rcp_b * (I.phi0 + dphi));
#pragma unroll
    for (int k = 0; k < 9; ++k) S.h[k][q] = rn ? hk[k] : real(0);
    (void)aphi; (void)sphi; (void)aT; (void)sT;
}

// Tile coordinates (hx, hy) of ring entry q: the row below, the row above,
// then the left and right columns.
template <int TX, int TY>
__device__ inline void ring_coords(int q, int& hx, int& hy)
{
    constexpr int PX = TX + 2;
    if (q < PX) { hx = q - 1; hy = -1; }
    else if (q < 2 * PX) { hx = q - PX - 1; hy = TY; }
    else {
        const int r = q - 2 * PX;
        hx = r < TY ? -1 : TX;
        hy = r < TY ? r : r - TY;
    }
}

// Loads the work-item's own node and fills the patch.  Returns whether the
// work-item's node lies in the lattice.  In interior tiles the first TX*TY
// ring entries go one per work-item, and their loads are issued together with
// the node's own, so that the workgroup waits for one memory round trip before
// the barrier, not two.
// TRIM: in a tile cut by the lattice's end, the stencils and the destination
// blend of its nodes read patch entries at most one column right of its last
// column and one row above its last row; the entries beyond are left unfilled
// (their loads would be wasted).  The potential form reads two columns
// further and does not trim.
template <typename real, int TX, int TY, bool EDGE, bool WHOLE, bool TRIM = false>
__device__ inline bool load_patch(const Inst<real>& I, int src, Patch<real, TX, TY>& S, int x0,
                                  int y0, real (&f)[9], real (&g)[9], real (&h)[9], real& jpx, real& jpy)
{
    using PT = Patch<real, TX, TY>;
    const int tid = threadIdx.x;
    const int lx = tid % TX, ly = tid / TX;
    const int gi = x0 + lx, gj = y0 + ly;
    const bool inside = WHOLE || (gi < I.nx && gj < I.ny);
    const int c = (ly + 1) * PT::PX + (lx + 1);
    // last patch column and row (tile coordinates) that any node of the tile reads
    const int lastx = WHOLE ? TX : (I.nx - x0 < TX ? I.nx - x0 : TX);
    const int lasty = WHOLE ? TY : (I.ny - y0 < TY ? I.ny - y0 : TY);
    auto used = [&](int hx, int hy) { return !TRIM || WHOLE || (hx <= lastx && hy <= lasty); };

    // ring entry `tid` of an interior tile (at most a periodic wrap): source
    // node and loads; edge tiles fill their ring after the node's own loads
    int rhx = 0, rhy = 0;
    if (!EDGE && tid < PT::NRING) ring_coords<TX, TY>(tid, rhx, rhy);
    const bool ring = !EDGE && tid < PT::NRING && used(rhx, rhy);
    int rc = 0;
    real rf[9], rh[9];
    if (ring) {
        const int hx = rhx, hy = rhy;
        rc = (hy + 1) * PT::PX + (hx + 1);
        const unsigned ridx = (unsigned)(wrap1(y0 + hy, I.ny) * I.pitch + wrap1(x0 + hx, I.nx));
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            rf[k] = ld(src_plane(I, src, kF + k), noff<real>(ridx));
            rh[k] = ld(src_plane(I, src, kH + k), noff<real>(ridx));
        }
    }
    if (inside) {
        const unsigned idx = (unsigned)(gj * I.pitch + gi);
        real sf = 0, sh = 0;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            f[k] = ld(src_plane(I, src, kF + k), noff<real>(idx));
            h[k] = ld(src_plane(I, src, kH + k), noff<real>(idx));
            g[k] = ld(src_plane(I, src, kG + k), noff<real>(idx));
        }
        // (phi u) of the previous level, needed after the barrier
        jpx = ld(to_global<const real>(I.jbase[0]), idx * (unsigned)sizeof(real));
        jpy = ld(to_global<const real>(I.jbase[1]), idx * (unsigned)sizeof(real));
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            sf += f[k];
            sh += h[k];
        }
        S.phi[c] = sf;
        S.T[c] = sh;
        S.irc[c] = recip(I.rcp_a + I.rcp_b * (I.phi0 + sf));
#pragma unroll
        for (int k = 0; k < 9; ++k) S.h[k][c] = h[k];
    } else if (used(lx, ly)) {
        fill_entry<real, EDGE>(I, src, S, c, gi, gj);
    }
    if (ring) {
        real sf = 0, sh = 0;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            sf += rf[k];
            sh += rh[k];
        }
        S.phi[rc] = sf;
        S.T[rc] = sh;
        S.irc[rc] = recip(I.rcp_a + I.rcp_b * (I.phi0 + sf));
#pragma unroll
        for (int k = 0; k < 9; ++k) S.h[k][rc] = rh[k];
    }
    // the remaining ring entries: all of an edge tile's, and those beyond one
    // per work-item
    for (int q = EDGE ? tid : tid + TX * TY; q < PT::NRING; q += TX * TY) {
        int hx, hy;
        ring_coords<TX, TY>(q, hx, hy);
        if (used(hx, hy)) fill_entry<real, EDGE>(I, src, S, (hy + 1) * PT::PX + (hx + 1), x0 + hx, y0 + hy);
    }
    __syncthreads();
    return inside;
}

// phi - phi0 at lattice point (gx, gy), at most two nodes outside the lattice,
// with the ghost rules applied.
template <typename real>
__device__ inline real phi_at(const Inst<real>& I, int src, int gx, int gy)
{
    int sx, sy;
    real aphi, sphi, aT, sT;
    const bool rn = resolve(I, gx, gy, sx, sy, aphi, sphi, aT, sT);
    const unsigned idx = (unsigned)(sy * I.pitch + sx);
    real sf = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) sf += ld(src_plane(I, src, kF + k), noff<real>(idx));
    (void)aT; (void)sT;
    return rn ? sf : aphi + sphi * sf;
}

// Potential form: mu_phi = phi^3 - phi - W^2 lap phi on the tile and its ring.
// The ring's Laplacian reads phi on a second ring (outer entries loaded here,
// ghost rules as for the first ring).  Every work-item of the workgroup calls
// this after load_patch (it synchronizes).
template <typename real, int TX, int TY>
__device__ inline void fill_mu(const Inst<real>& I, int src, const Patch<real, TX, TY>& S, PotLDS<real, TX, TY>& Q,
                               int x0, int y0)
{
    constexpr int PX = TX + 2, PY = TY + 2, QX = TX + 4, QY = TY + 4;
    for (int q = threadIdx.x; q < QX * QY; q += TX * TY) {
        const int qx = q % QX, qy = q / QX;
        const bool inner = qx >= 1 && qx <= PX && qy >= 1 && qy <= PY;
        Q.phw[q] = inner ? S.phi[(qy - 1) * PX + (qx - 1)] : phi_at(I, src, x0 + qx - 2, y0 + qy - 2);
    }
    __syncthreads();
    for (int q = threadIdx.x; q < PX * PY; q += TX * TY) {
        const int c = (q / PX + 1) * QX + (q % PX + 1);
        const real pc = Q.phw[c];
        const real lap = real(2.0 / 3.0) * ((Q.phw[c + 1] + Q.phw[c - 1]) + (Q.phw[c + QX] + Q.phw[c - QX]) - real(4) * pc)
                       + real(1.0 / 6.0) * ((Q.phw[c + QX + 1] + Q.phw[c + QX - 1]) + (Q.phw[c - QX - 1] + Q.phw[c - QX + 1])
                                            - real(4) * pc);
        const real phi = I.phi0 + pc;
        const real pm1 = (I.phi0 - real(1)) + pc;
        Q.mu[q] = pm1 * (phi + real(1)) * phi - I.W2 * lap;
    }
    __syncthreads();
}

// Patch offsets of the eight neighbours of an entry, by direction k = 1..8:
// fixed for a TX x TY tile patch of row length PX, per node for a run.
template <int PX>
struct GridNb {
    __device__ static constexpr int at(int k) { return cy(k) * PX + cx(k); }
};
struct RunNb {
    int o[9];
    __device__ int at(int k) const { return o[k]; }
};

template <typename real>
struct Macro {
    real dphi, phi, theta;
    real gpx, gpy, gtx, gty;
    real rho, ux, uy, p, Fx, Fy, grx, gry, irho;
};

// Pass-1 quantities of one node from the patch and its own g_i.  POT: the
// lattice may use the potential form of the capillary force, with mu_phi of the
// patch in smu.
template <typename real, typename NB, bool POT = false>
__device__ inline Macro<real> node_macros(const Inst<real>& I, const real* __restrict__ sphi,
                                          const real* __restrict__ sT, int c, const NB& nb, const real (&g)[9],
                                          const real* __restrict__ smu = nullptr)
{
    Macro<real> m;
    const real pc = sphi[c];
    const real pE = sphi[c + nb.at(1)], pW = sphi[c + nb.at(3)], pN = sphi[c + nb.at(2)], pS = sphi[c + nb.at(4)];
    const real pNE = sphi[c + nb.at(5)], pNW = sphi[c + nb.at(6)], pSW = sphi[c + nb.at(7)], pSE = sphi[c + nb.at(8)];
    const real tE = sT[c + nb.at(1)], tW = sT[c + nb.at(3)], tN = sT[c + nb.at(2)], tS = sT[c + nb.at(4)];
    const real tNE = sT[c + nb.at(5)], tNW = sT[c + nb.at(6)], tSW = sT[c + nb.at(7)], tSE = sT[c + nb.at(8)];
    const real third = real(1.0 / 3.0), twelfth = real(1.0 / 12.0);
    // grad psi = 3 sum w_i c_i psi(x + c_i); lap psi = 6 sum_{i>0} w_i (psi(x + c_i) - psi(x))
    m.gpx = third * (pE - pW) + twelfth * ((pNE - pNW) + (pSE - pSW));
    m.gpy = third * (pN - pS) + twelfth * ((pNE + pNW) - (pSW + pSE));
    const real lap = real(2.0 / 3.0) * ((pE + pW) + (pN + pS) - real(4) * pc)
                   + real(1.0 / 6.0) * ((pNE + pNW) + (pSW + pSE) - real(4) * pc);
    m.gtx = third * (tE - tW) + twelfth * ((tNE - tNW) + (tSE - tSW));
    m.gty = third * (tN - tS) + twelfth * ((tNE + tNW) - (tSW + tSE));

    m.dphi = pc;
    m.phi = I.phi0 + pc;
    m.theta = sT[c];
    const real phi = m.phi;
    m.rho = I.rho_a + I.rho_b * phi;
    m.irho = recip(m.rho);
    m.grx = I.rho_b * m.gpx;
    m.gry = I.rho_b * m.gpy;
    // chemical potential phi^3 - phi - W^2 lap phi, written so that phi - 1 is exact near phi0 = 1
    const real pm1 = (I.phi0 - real(1)) + pc;
    const real mu_phi = pm1 * (phi + real(1)) * phi - I.W2 * lap;
    // sigma(T) and grad sigma = sigma'(T) grad T
    const real dT = I.dTref + m.theta;
    const real sig = I.sigma_ref + dT * (I.sigma_T + real(0.5) * I.sigma_TT * dT);
    const real dsig = I.sigma_T + I.sigma_TT * dT;
    const real gsx = dsig * m.gtx, gsy = dsig * m.gty;
    // F_s = 3 sqrt2 W/4 [|grad phi|^2 grad sigma - (grad sigma . grad phi) grad phi + sigma/W^2 mu_phi grad phi]
    const real g2 = m.gpx * m.gpx + m.gpy * m.gpy;
    const real sdp = gsx * m.gpx + gsy * m.gpy;
    if (POT && I.force_form == 1) {
        // potential form: -phi grad mu_phi in place of mu_phi grad phi
        const real mE = smu[c + nb.at(1)], mW = smu[c + nb.at(3)], mN = smu[c + nb.at(2)], mS = smu[c + nb.at(4)];
        const real mNE = smu[c + nb.at(5)], mNW = smu[c + nb.at(6)], mSW = smu[c + nb.at(7)], mSE = smu[c + nb.at(8)];
        const real gmx = third * (mE - mW) + twelfth * ((mNE - mNW) + (mSE - mSW));
        const real gmy = third * (mN - mS) + twelfth * ((mNE + mNW) - (mSW + mSE));
        const real sp = sig * I.inv_W2 * phi;
        m.Fx = I.pref * (g2 * gsx - sdp * m.gpx - sp * gmx) + I.Gx;
        m.Fy = I.pref * (g2 * gsy - sdp * m.gpy - sp * gmy) + I.Gy;
    } else {
        const real cap = sig * I.inv_W2 * mu_phi;
        m.Fx = I.pref * (g2 * gsx + (cap - sdp) * m.gpx) + I.Gx;
        m.Fy = I.pref * (g2 * gsy + (cap - sdp) * m.gpy) + I.Gy;
    }
    // rho u = sum c_i g_i + F/2
    const real mx = (g[1] - g[3]) + (g[5] - g[6]) + (g[8] - g[7]);
    const real my = (g[2] - g[4]) + (g[5] + g[6]) - (g[7] + g[8]);
    m.ux = (mx + real(0.5) * m.Fx) * m.irho;
    m.uy = (my + real(0.5) * m.Fy) * m.irho;
    // p = c_s^2/(1 - w_0) [sum_{i>0} g_i + u.grad rho/2 + rho s_0(u)], s_0 = -w_0 |u|^2 / (2 c_s^2)
    const real sg = ((g[1] + g[2]) + (g[3] + g[4])) + ((g[5] + g[6]) + (g[7] + g[8]));
    const real uu = m.ux * m.ux + m.uy * m.uy;
    m.p = real(0.6) * (sg + real(0.5) * (m.ux * m.grx + m.uy * m.gry) - real(2.0 / 3.0) * m.rho * uu);
    return m;
}

// Streaming destination of direction k from (gi, gj): returns true and the
// destination index if it stays in the lattice (after periodic wrap);
// otherwise returns false and the side whose rule applies.
template <typename real, bool EDGE>
__device__ inline bool dest(const Inst<real>& I, int gi, int gj, int k, unsigned& idx, int& side)
{
    if (!EDGE) {
        idx = (unsigned)(wrap1(gj + cy(k), I.ny) * I.pitch + wrap1(gi + cx(k), I.nx));
        side = 0;
        return true;
    }
    int ti = gi + cx(k), tj = gj + cy(k);
    bool ox = false, oy = false;
    int sxs = 0, sys = 2;
    if (ti < 0) { sxs = 0; if (I.bc[0] == BC_PERIODIC) ti += I.nx; else ox = true; }
    else if (ti >= I.nx) { sxs = 1; if (I.bc[1] == BC_PERIODIC) ti -= I.nx; else ox = true; }
    if (tj < 0) { sys = 2; if (I.bc[2] == BC_PERIODIC) tj += I.ny; else oy = true; }
    else if (tj >= I.ny) { sys = 3; if (I.bc[3] == BC_PERIODIC) tj -= I.ny; else oy = true; }
    if (!ox && !oy) {
        idx = (unsigned)(tj * I.pitch + ti);
        return true;
    }
    if (ox && oy) {
        const int bx = I.bc[sxs], by = I.bc[sys];
        const int px = (bx == BC_WALL_T || bx == BC_WALL_ADIABATIC) ? 2 : (bx == BC_INLET ? 1 : 0);
        const int py = (by == BC_WALL_T || by == BC_WALL_ADIABATIC) ? 2 : (by == BC_INLET ? 1 : 0);
        side = px > py ? sxs : sys;
    } else {
        side = ox ? sxs : sys;
    }
    return false;
}

// Collision quantities of one node beyond its macros.
template <typename real>
struct Pre {
    real inv_tau_g, fac_g, inv_tau_h, inv_tau_gm, fac_gm, inv_tau_hp;
    real ax, ay;  // R_i = w_i c_i . (ax, ay)
    real Fhat, uu, p3;
};

// Relaxation rates, the Allen-Cahn source vector and the thermal source of a
// node; jx, jy return phi u, the next level's previous value.
template <typename real, bool TRT>
__device__ __forceinline__ Pre<real> pre_collide(const Inst<real>& I, const Macro<real>& m, const real (&f)[9],
                                                 const real (&h)[9], real jpx, real jpy, real& jx, real& jy)
{
    Pre<real> q;
    const real phi = m.phi, ux = m.ux, uy = m.uy;
    const real mu = I.mu_a + I.mu_b * phi;
    const real lam = I.lam_a + I.lam_b * phi;
    const real rcp = I.rcp_a + I.rcp_b * phi;
    // mu = rho c_s^2 (tau_g - 1/2), lambda = c_s^2 (tau_h - 1/2)
    q.inv_tau_g = m.rho * recip(real(0.5) * m.rho + real(3) * mu);
    q.fac_g = real(1) - real(0.5) * q.inv_tau_g;
    const real tau_h = real(0.5) + real(3) * lam;
    q.inv_tau_h = recip(tau_h);
    // two relaxation times: (tau+ - 1/2)(tau- - 1/2) = trt_magic; the NS LBE's
    // even part and the thermal LBE's odd part keep the times above
    q.inv_tau_gm = 0;
    q.fac_gm = 0;
    q.inv_tau_hp = 0;
    if (TRT) {
        const real tau_g = real(1) / q.inv_tau_g;
        q.inv_tau_gm = recip(real(0.5) + I.trt_magic * recip(tau_g - real(0.5)));
        q.fac_gm = real(1) - real(0.5) * q.inv_tau_gm;
        q.inv_tau_hp = recip(real(0.5) + I.trt_magic * recip(tau_h - real(0.5)));
    }

    // time derivative of phi u by the first-order Euler scheme
    jx = phi * ux;
    jy = phi * uy;
    const real djx = jx - jpx, djy = jy - jpy;

    // Allen-Cahn source: unit normal from v = sum c_i (f_i - f_i^eq) + dt(phi u)/2, n = -v/|v|
    real nxv = 0, nyv = 0;
    if (I.grad_mode == 0) {
        const real vx = ((f[1] - f[3]) + (f[5] - f[6]) + (f[8] - f[7])) - jx + real(0.5) * djx;
        const real vy = ((f[2] - f[4]) + (f[5] + f[6]) - (f[7] + f[8])) - jy + real(0.5) * djy;
        const real vn2 = vx * vx + vy * vy;
        if (has_direction(vn2)) {
            const real iv = rsq(vn2);
            nxv = -vx * iv;
            nyv = -vy * iv;
        }
    } else {
        const real gn2 = m.gpx * m.gpx + m.gpy * m.gpy;
        if (has_direction(gn2)) {
            const real ig = rsq(gn2);
            nxv = m.gpx * ig;
            nyv = m.gpy * ig;
        }
    }
    const real pm1 = (I.phi0 - real(1)) + m.dphi;
    const real lamc = -pm1 * (phi + real(1)) * I.inv_s2W;  // (1 - phi^2)/(sqrt2 W)
    q.ax = real(3) * djx + lamc * nxv;                      // R_i = w_i c_i . (3 dt(phi u) + lamc n)
    q.ay = real(3) * djy + lamc * nyv;

    // thermal source: grad T from the first moment of h (or the stencil), Fhat = -rho c_p u . grad T
    real tgx, tgy;
    if (I.grad_mode == 0) {
        const real hx = (h[1] - h[3]) + (h[5] - h[6]) + (h[8] - h[7]);
        const real hy = (h[2] - h[4]) + (h[5] + h[6]) - (h[7] + h[8]);
        tgx = real(-3) * hx * q.inv_tau_h;
        tgy = real(-3) * hy * q.inv_tau_h;
    } else {
        tgx = m.gtx;
        tgy = m.gty;
    }
    q.Fhat = -rcp * (ux * tgx + uy * tgy);
    q.uu = ux * ux + uy * uy;
    q.p3 = real(3) * m.p;
    return q;
}

// Post-collision values of direction k of one node (Eq. 14, the NS LBE and the
// collision part of Eq. 28).  Directions 1..8 come first and accumulate their
// changes in df, dh; the rest populations (k = 0) then take the balance:
// f*_0 = f_0 + sum_{i>0} (f_i - f*_i), h*_0 = h_0 + Fhat + sum_{i>0} (h_i - h*_i),
// equal to their BGK values in real arithmetic (sum_i f*_i = sum_i f_i,
// sum_i h*_i = sum_i h_i + Fhat); this keeps the stored update mass- and
// heat-neutral up to one rounding.  Otherwise each node relaxes toward w_i
// times its rounded moment, and identical bulk nodes round alike, so FP32
// storage drifts linearly in time.
template <typename real, bool TRT>
__device__ __forceinline__ void collide_dir(const Inst<real>& I, const Macro<real>& m, const Pre<real>& q, int k,
                                            const real (&f)[9], const real (&g)[9], const real (&h)[9], real& df,
                                            real& dh, real& fsk, real& gsk, real& hsk)
{
    const real w = wgt<real>(k);
    const real cu = real(cx(k)) * m.ux + real(cy(k)) * m.uy;
    // NS LBE: g^eq = 3 p (w_i - delta_i0) + rho s_i(u); G_i = w_i [3 c_i.F + 3 (c_i.u)(c_i.grad rho)]
    const real si = w * (real(3) * cu + real(4.5) * cu * cu - real(1.5) * q.uu);
    const real geq = (k == 0 ? q.p3 * (w - real(1)) : q.p3 * w) + m.rho * si;
    const real cF = real(cx(k)) * m.Fx + real(cy(k)) * m.Fy;
    const real cg = real(cx(k)) * m.grx + real(cy(k)) * m.gry;
    const real Gi = w * real(3) * (cF + cu * cg);
    if (!TRT) {
        gsk = g[k] - (g[k] - geq) * q.inv_tau_g + q.fac_g * Gi;
    } else {
        // even and odd parts under c_i -> -c_i of g_i, g_i^eq and G_i
        const int kb = opp(k);
        const real gp = real(0.5) * (g[k] + g[kb]), gm = real(0.5) * (g[k] - g[kb]);
        const real ep = (k == 0 ? q.p3 * (w - real(1)) : q.p3 * w) + m.rho * w * (real(4.5) * cu * cu - real(1.5) * q.uu);
        const real em = m.rho * w * real(3) * cu;
        const real Gp = w * real(3) * (cu * cg), Gm = w * real(3) * cF;
        gsk = g[k] - (gp - ep) * q.inv_tau_g - (gm - em) * q.inv_tau_gm + q.fac_g * Gp + q.fac_gm * Gm;
    }
    if (k == 0) {
        fsk = f[0] + df;
        hsk = (h[0] + q.Fhat) + dh;
    } else {
        // Eq. 14: f* = f - (f - f^eq)/tau_phi + (1 - 1/(2 tau_phi)) R_i
        const real feq = w * (m.dphi + real(3) * m.phi * cu);
        const real Ri = w * (real(cx(k)) * q.ax + real(cy(k)) * q.ay);
        fsk = f[k] - (f[k] - feq) * I.inv_tau_phi + I.fac_phi * Ri;
        // Eq. 28 collision part: h - (h - w_i T)/tau_h + w_i Fhat; with two
        // relaxation times the odd part (conduction) keeps tau_h
        if (!TRT) {
            hsk = h[k] - (h[k] - w * m.theta) * q.inv_tau_h + w * q.Fhat;
        } else {
            const int kb = opp(k);
            const real hp = real(0.5) * (h[k] + h[kb]), hm = real(0.5) * (h[k] - h[kb]);
            hsk = h[k] - (hp - w * m.theta) * q.inv_tau_hp - hm * q.inv_tau_h + w * q.Fhat;
        }
        df += f[k] - fsk;
        dh += h[k] - hsk;
    }
}

// Collision and push streaming of the node (gi, gj) at patch entry c, whose
// populations are f, g, h.  The thermal update at the destination y = x + c_i
// is h_i(y, t+1) = [h*_i(x) + (rho c_p(y) - 1) h_i(y, t)] / rho c_p(y).
// Each direction is stored as soon as it is collided.
template <typename real, bool EDGE, bool TRT, bool POT, typename P, typename NB>
__device__ __forceinline__ void node_update(const Inst<real>& I, const P& S, const NB& nb, const real* smu, int gi,
                                            int gj, int c, int dst, const real (&f)[9], const real (&g)[9],
                                            const real (&h)[9], real jpx, real jpy)
{
    const unsigned own = (unsigned)(gj * I.pitch + gi);
    const gptr<real> Jx = to_global(I.jbase[0]), Jy = to_global(I.jbase[1]);
    // destination rows and columns of the interior path (periodic wrap only)
    unsigned drow[3] = {0, 0, 0}, dcol[3] = {0, 0, 0};
    if (!EDGE) {
        drow[0] = (unsigned)(wrap1(gj - 1, I.ny) * I.pitch);
        drow[1] = (unsigned)(gj * I.pitch);
        drow[2] = (unsigned)(wrap1(gj + 1, I.ny) * I.pitch);
        dcol[0] = (unsigned)wrap1(gi - 1, I.nx);
        dcol[1] = (unsigned)gi;
        dcol[2] = (unsigned)wrap1(gi + 1, I.nx);
    }

    const Macro<real> m = node_macros<real, NB, POT>(I, S.phi, S.T, c, nb, g, smu);
    real jx, jy;
    const Pre<real> q = pre_collide<real, TRT>(I, m, f, h, jpx, jpy, jx, jy);
    st(Jx, own * (unsigned)sizeof(real), jx);
    st(Jy, own * (unsigned)sizeof(real), jy);

    real df = 0, dh = 0;
#pragma unroll
    for (int kk = 1; kk <= 9; ++kk) {
        const int k = kk % 9;  // directions 1..8, then the rest population
        real fsk, gsk, hsk;
        collide_dir<real, TRT>(I, m, q, k, f, g, h, df, dh, fsk, gsk, hsk);
        unsigned di = 0;
        int side = 0;
        bool in_lattice = true;
        if (EDGE) in_lattice = dest<real, EDGE>(I, gi, gj, k, di, side);
        else di = drow[cy(k) + 1] + dcol[cx(k) + 1];
        if (in_lattice) {
            const int cd = c + nb.at(k);
            st(dst_plane(I, dst, kF + k), noff<real>(di), (real)(fsk));
            st(dst_plane(I, dst, kG + k), noff<real>(di), (real)(gsk));
            const real hold = S.h[k][cd];
            st(dst_plane(I, dst, kH + k), noff<real>(di), (real)(hold + (hsk - hold) * S.irc[cd]));
        } else if (EDGE) {
            const int kb = opp(k);
            const int bc = I.bc[side];
            const real w = wgt<real>(k);
            const real cu = real(cx(k)) * m.ux + real(cy(k)) * m.uy;
            // crossing point of the link: s = s2 / 2 along the side
            const int s2 = side < 2 ? 2 * gj + cy(k) : 2 * gi + cx(k);
            real fb, gb, hb;
            if (bc == BC_WALL_T || bc == BC_WALL_ADIABATIC) {
                // halfway bounce-back; anti-bounce-back for a Dirichlet temperature
                fb = fsk;
                gb = gsk;
                hb = bc == BC_WALL_T ? -hsk + real(2) * w * wall_T(I, side, s2) : hsk;
            } else if (bc == BC_INLET) {
                // anti-bounce-back for phi and T, moving-wall bounce-back for u
                const real H = side < 2 ? real(I.ny) : real(I.nx);
                const real sp = real(0.5) * real(s2 + 1);
                const real un = real(6) * I.u_in * sp * (H - sp) / (H * H);
                const real uix = side == 0 ? un : (side == 1 ? -un : real(0));
                const real uiy = side == 2 ? un : (side == 3 ? -un : real(0));
                fb = -fsk + real(2) * w * I.phi_in_d;
                gb = gsk - real(6) * w * m.rho * (real(cx(k)) * uix + real(cy(k)) * uiy);
                hb = -hsk + real(2) * w * I.T_in_d;
            } else {  // outlet: anti-bounce-back at p = 0 with the node's own u, phi, T
                fb = -fsk + real(2) * w * m.dphi;
                gb = -gsk + real(2) * w * m.rho * (real(4.5) * cu * cu - real(1.5) * q.uu);
                hb = -hsk + real(2) * w * m.theta;
            }
            st(dst_plane(I, dst, kF + kb), noff<real>(own), (real)(fb));
            st(dst_plane(I, dst, kG + kb), noff<real>(own), (real)(gb));
            const real hold = S.h[kb][c];
            st(dst_plane(I, dst, kH + kb), noff<real>(own), (real)(hold + (hb - hold) * S.irc[c]));
        }
    }
}

// Slots that no node owns: the few between a row's last node and the next
// row's first (rows start on aligned boundaries) and the lattice's tail up to
// the end of its last cache line.  Left unwritten, they would leave those
// lines of every population run partly written each step, and the memory side
// would have to merge them with their old contents.  A work-item whose node
// lies beyond its row stores zeros into such slots of the next level.  Nothing
// reads them.
template <typename real>
__device__ inline void pad_line(const Inst<real>& I, int dst, int gi, int gj)
{
    constexpr unsigned line_nodes = 128 / (unsigned)sizeof(real);
    if (gj >= I.ny || gi < I.nx) return;
    const unsigned nn = (unsigned)I.pitch * (unsigned)I.ny;
    const unsigned own = (unsigned)gj * (unsigned)I.pitch + (unsigned)gi;
    const bool gap = gi < I.pitch;
    const bool tail = gj == I.ny - 1 && own < (nn + line_nodes - 1) / line_nodes * line_nodes;
    if (!gap && !tail) return;
#pragma unroll
    for (int q = 0; q < kPlanes; ++q) st(dst_plane(I, dst, q), noff<real>(own), real(0));
    st(to_global(I.jbase[0]), own * (unsigned)sizeof(real), real(0));
    st(to_global(I.jbase[1]), own * (unsigned)sizeof(real), real(0));
}

// One node per work-item.  POT (with QT = PotLDS): the lattice may use the
// potential form of the capillary force.
template <typename real, int TX, int TY, bool EDGE, bool WHOLE, bool TRT, bool POT = false, typename QT = NoPot>
__device__ __forceinline__ void tile_step(const Inst<real>& I, int x0, int y0, int src, Patch<real, TX, TY>& S,
                                          QT& Q)
{
    real f[9], g[9], h[9], jpx = 0, jpy = 0;
    const bool inside = load_patch<real, TX, TY, EDGE, WHOLE, !POT>(I, src, S, x0, y0, f, g, h, jpx, jpy);
    const real* smu = nullptr;
    if constexpr (POT) {
        // uniform branch: every work-item reaches the barriers of fill_mu
        if (I.force_form == 1) fill_mu<real, TX, TY>(I, src, S, Q, x0, y0);
        smu = Q.mu;
    }
    const int tid = threadIdx.x;
    if (!inside) {
        if (!WHOLE) pad_line(I, src ^ 1, x0 + tid % TX, y0 + tid / TX);
        return;
    }
    constexpr int PX = Patch<real, TX, TY>::PX;
    const int c = (tid / TX + 1) * PX + (tid % TX + 1);
    node_update<real, EDGE, TRT, POT>(I, S, GridNb<PX>{}, smu, x0 + tid % TX, y0 + tid / TX, c, src ^ 1, f, g, h, jpx,
                                      jpy);
}

// Interior tiles take the wrap-only path; a whole one needs no per-node
// inside test (a partial one, cut by the lattice's end in a periodic
// direction, does).
template <typename real, int TX, int TY, bool TRT>
__device__ __forceinline__ void tile_any(const Inst<real>& I, const Tile& tl, int src, Patch<real, TX, TY>& S)
{
    NoPot none;
    if (tl.flags & kTileInterior) {
        if (tl.flags & kTileWhole) tile_step<real, TX, TY, false, true, TRT>(I, tl.x0, tl.y0, src, S, none);
        else tile_step<real, TX, TY, false, false, TRT>(I, tl.x0, tl.y0, src, S, none);
    } else {
        tile_step<real, TX, TY, true, false, TRT>(I, tl.x0, tl.y0, src, S, none);
    }
}

// Dispatch for a launch that may hold lattices with the potential form of the
// capillary force (their second ring is always resolved by the general ghost
// rules).  In FP32 every tile takes the general path: with the interior path
// beside it the kernel needs more than 128 VGPRs and loses a wave per SIMD
// (measured 18% slower); in FP64 the interior path gains 2-8%.
template <typename real, int TX, int TY, bool TRT>
__device__ __forceinline__ void tile_pot(const Inst<real>& I, const Tile& tl, int src, Patch<real, TX, TY>& S,
                                         PotLDS<real, TX, TY>& Q)
{
    if (sizeof(real) == 4) {
        tile_step<real, TX, TY, true, false, TRT, true>(I, tl.x0, tl.y0, src, S, Q);
    } else if (tl.flags & kTileInterior) {
        if (tl.flags & kTileWhole) tile_step<real, TX, TY, false, true, TRT, true>(I, tl.x0, tl.y0, src, S, Q);
        else tile_step<real, TX, TY, false, false, TRT, true>(I, tl.x0, tl.y0, src, S, Q);
    } else {
        tile_step<real, TX, TY, true, false, TRT, true>(I, tl.x0, tl.y0, src, S, Q);
    }
}

template <typename real, int TX, int TY>
__device__ __forceinline__ bool load_any(const Inst<real>& I, const Tile& tl, int src, Patch<real, TX, TY>& S,
                                         real (&f)[9], real (&g)[9], real (&h)[9])
{
    real jpx, jpy;  // unused here: the loads are dropped
    if (tl.flags & kTileInterior) {
        if (tl.flags & kTileWhole)
            return load_patch<real, TX, TY, false, true>(I, src, S, tl.x0, tl.y0, f, g, h, jpx, jpy);
        return load_patch<real, TX, TY, false, false>(I, src, S, tl.x0, tl.y0, f, g, h, jpx, jpy);
    }
    return load_patch<real, TX, TY, true, false>(I, src, S, tl.x0, tl.y0, f, g, h, jpx, jpy);
}

// ---- runs ----
// A run is RN consecutive nodes of a lattice in x-fastest order (node
// number n = y nx + x), one per work-item, so rows of any width leave no
// work-item idle.  Used for lattices periodic in x with
// kRunMinNx <= nx <= kRunMaxNx.  The patch of a run starting at n0 is the
// window of node numbers n0 - nx - 1 ... n0 + RN + nx (window slot
// w = m - n0 + nx + 1 for node number m), which holds every neighbour of the
// run's nodes in the rows below and above.  A neighbour across the periodic x
// boundary sits nx - 1 or nx + 1 slots away from where it would be without the
// wrap; the two that can fall outside the window, (0, y - 1) of the first
// node with x = nx - 1 and (nx - 1, y + 1) of the last node with x = 0, get
// slots of their own at the end.  Slots of rows -1 and ny are the ghosts of
// the boundary rules (runs holding no node of the first or last row never
// read them).  The four corner ghosts (-1, -1), (nx, -1), (-1, ny), (nx, ny)
// also get slots of their own: a wall's rule is evaluated at the unwrapped
// coordinate along the wall (a Dirichlet temperature at -1 or nx), as for
// every other ghost of a tile's ring.
template <typename real, int RN>
struct RunPatch {
    static constexpr int NW = RN + 2 * kRunMaxNx + 8;
    static constexpr int GLO = NW - 6, GHI = NW - 5;
    static constexpr int CSW = NW - 4, CSE = NW - 3, CNW = NW - 2, CNE = NW - 1;
    real phi[NW];
    real T[NW];
    real irc[NW];
    real h[9][NW];
};

template <typename real, int TX, int TY>
union StepLDS {
    Patch<real, TX, TY> tile;
    RunPatch<real, TX * TY> run;
};

// Window slot and lattice point of ring entry q of the run from n0 (q in
// [0, 2 nx + 4), and in EDGE runs also [2 nx + 4, 2 nx + 8): the slots below
// the run, those above it, the two wrap slots, then the four corner ghosts);
// yl is the row of the run's last node.  Returns whether a node of the run may
// read the entry: EDGE runs read rows -1 .. ny, interior runs rows 0 .. ny - 1
// only.
template <bool EDGE, int RN>
__device__ inline bool run_ring(int q, int n0, int nx, int ny, int yl, int& w, int& gx, int& gy)
{
    using RP = RunPatch<float, RN>;  // slot numbers do not depend on the word size
    if (EDGE && q >= 2 * nx + 4) {
        const int k = q - (2 * nx + 4);
        w = RP::CSW + k;
        gx = (k & 1) ? nx : -1;
        gy = (k & 2) ? ny : -1;
        return true;
    }
    if (q < 2 * nx + 2) {
        w = q < nx + 1 ? q : q + RN;
        const int m = n0 - nx - 1 + w;
        if (m < -nx) return false;
        gy = (m + nx) / nx - 1;
        gx = m - gy * nx;
        return EDGE ? gy <= ny : (gy >= 0 && gy < ny);
    }
    const int y0 = n0 / nx, x0 = n0 - y0 * nx;
    if (q == 2 * nx + 2) {
        // (0, y0 - 1): south-east neighbour of the first node with x = nx - 1,
        // outside the window when that node is among the first nx - 2
        w = RP::GLO;
        gx = 0;
        gy = y0 - 1;
        return x0 >= 2;
    }
    // (nx - 1, yl + 1): north-west neighbour of the last node with x = 0 (in
    // row yl), outside the window when that node is among the last nx - 2
    // slots of the run
    w = RP::GHI;
    gx = nx - 1;
    gy = yl + 1;
    return yl * nx - n0 >= RN - nx + 2;
}

// Plain fill of a run window slot from lattice point (gx, gy) inside the lattice.
template <typename real>
__device__ inline void run_load_entry(const Inst<real>& I, int src, int gx, int gy, real (&rf)[9], real (&rh)[9])
{
    const unsigned idx = (unsigned)(gy * I.pitch + gx);
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        rf[k] = ld(src_plane(I, src, kF + k), noff<real>(idx));
        rh[k] = ld(src_plane(I, src, kH + k), noff<real>(idx));
    }
}

template <typename real, int RN>
__device__ inline void run_store_entry(RunPatch<real, RN>& R, const Inst<real>& I, int w, const real (&rf)[9],
                                       const real (&rh)[9])
{
    real sf = 0, sh = 0;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        sf += rf[k];
        sh += rh[k];
    }
    R.phi[w] = sf;
    R.T[w] = sh;
    R.irc[w] = recip(I.rcp_a + I.rcp_b * (I.phi0 + sf));
#pragma unroll
    for (int k = 0; k < 9; ++k) R.h[k][w] = rh[k];
}

// Loads the work-item's own node of the run from n0 and fills the window.
// Returns whether the node lies in the lattice; (x, y) its coordinates.  In
// interior runs the first RN ring entries go one per work-item and their
// loads are issued together with the node's own.
template <typename real, bool EDGE, int RN>
__device__ inline bool load_run(const Inst<real>& I, int src, RunPatch<real, RN>& R, int n0, int& x, int& y,
                                real (&f)[9], real (&g)[9], real (&h)[9], real& jpx, real& jpy)
{
    const int nx = I.nx, ny = I.ny, nn = nx * ny;
    const int t = threadIdx.x;
    const int n = n0 + t;
    const bool inside = n < nn;
    y = n / nx;
    x = n - y * nx;
    const int c = t + nx + 1;
    const int nring = 2 * nx + (EDGE ? 8 : 4);
    const int last = (n0 + RN < nn ? n0 + RN : nn) - 1;
    const int yl = last / nx;

    int rw = 0, rgx = 0, rgy = 0;
    const bool ring = !EDGE && t < nring && run_ring<false, RN>(t, n0, nx, ny, yl, rw, rgx, rgy);
    real rf[9], rh[9];
    if (ring) run_load_entry(I, src, rgx, rgy, rf, rh);
    if (inside) {
        const unsigned idx = (unsigned)(y * I.pitch + x);
        real sf = 0, sh = 0;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            f[k] = ld(src_plane(I, src, kF + k), noff<real>(idx));
            h[k] = ld(src_plane(I, src, kH + k), noff<real>(idx));
            g[k] = ld(src_plane(I, src, kG + k), noff<real>(idx));
        }
        jpx = ld(to_global<const real>(I.jbase[0]), idx * (unsigned)sizeof(real));
        jpy = ld(to_global<const real>(I.jbase[1]), idx * (unsigned)sizeof(real));
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            sf += f[k];
            sh += h[k];
        }
        R.phi[c] = sf;
        R.T[c] = sh;
        R.irc[c] = recip(I.rcp_a + I.rcp_b * (I.phi0 + sf));
#pragma unroll
        for (int k = 0; k < 9; ++k) R.h[k][c] = h[k];
    } else if (EDGE && y == ny) {
        // beyond the lattice's last node: the slot is a ghost of row ny
        fill_entry<real, true>(I, src, R, c, x, y);
    }
    if (ring) run_store_entry(R, I, rw, rf, rh);
    for (int q = EDGE ? t : t + RN; q < nring; q += RN) {
        int w, gx, gy;
        if (!run_ring<EDGE, RN>(q, n0, nx, ny, yl, w, gx, gy)) continue;
        if (EDGE) {
            fill_entry<real, true>(I, src, R, w, gx, gy);
        } else {
            real qf[9], qh[9];
            run_load_entry(I, src, gx, gy, qf, qh);
            run_store_entry(R, I, w, qf, qh);
        }
    }
    __syncthreads();
    return inside;
}

// Slots between a row's last node and the next row's first (FP32 rows start
// on 64-byte boundaries) and the lattice's tail up to the end of its last cache
// line: the row's last nodes store zeros into them in the next level, so no
// line is left partly written.
template <typename real>
__device__ inline void run_pad(const Inst<real>& I, int dst, int x, int y)
{
    constexpr unsigned line_nodes = 128 / (unsigned)sizeof(real);
    int ext = I.pitch - I.nx;
    if (y == I.ny - 1) {
        const unsigned nn = (unsigned)I.pitch * (unsigned)I.ny;
        ext += (int)((nn + line_nodes - 1) / line_nodes * line_nodes - nn);
    }
    if (ext == 0 || x < I.nx - ext) return;
    const unsigned own = (unsigned)(y * I.pitch + I.nx + (x - (I.nx - ext)));
#pragma unroll
    for (int q = 0; q < kPlanes; ++q) st(dst_plane(I, dst, q), noff<real>(own), real(0));
    st(to_global(I.jbase[0]), own * (unsigned)sizeof(real), real(0));
    st(to_global(I.jbase[1]), own * (unsigned)sizeof(real), real(0));
}

template <typename real, bool EDGE, bool TRT, int RN>
__device__ __forceinline__ void run_step(const Inst<real>& I, int n0, int src, RunPatch<real, RN>& R)
{
    using RP = RunPatch<real, RN>;
    real f[9], g[9], h[9], jpx = 0, jpy = 0;
    int x, y;
    const bool inside = load_run<real, EDGE, RN>(I, src, R, n0, x, y, f, g, h, jpx, jpy);
    if (!inside) return;
    const int nx = I.nx, t = threadIdx.x, c = t + nx + 1;
    const bool xl = x == 0, xr = x == nx - 1;
    // corner ghosts (only EDGE runs hold nodes of the first or last row)
    const bool bot = EDGE && y == 0, top = EDGE && y == I.ny - 1;
    RunNb nb;
    nb.o[0] = 0;
    nb.o[1] = xr ? 1 - nx : 1;
    nb.o[2] = nx;
    nb.o[3] = xl ? nx - 1 : -1;
    nb.o[4] = -nx;
    nb.o[5] = xr ? (top ? RP::CNE - c : 1) : nx + 1;
    nb.o[6] = xl ? (top ? RP::CNW - c : (t < RN - nx + 2 ? 2 * nx - 1 : RP::GHI - c)) : nx - 1;
    nb.o[7] = xl ? (bot ? RP::CSW - c : -1) : -nx - 1;
    nb.o[8] = xr ? (bot ? RP::CSE - c : (t >= nx - 2 ? 1 - 2 * nx : RP::GLO - c)) : 1 - nx;
    run_pad(I, src ^ 1, x, y);
    node_update<real, EDGE, TRT, false>(I, R, nb, nullptr, x, y, c, src ^ 1, f, g, h, jpx, jpy);
}

template <typename real, bool TRT, int RN>
__device__ __forceinline__ void run_any(const Inst<real>& I, const Tile& tl, int src, RunPatch<real, RN>& R)
{
    if (tl.flags & kTileInterior) run_step<real, false, TRT, RN>(I, tl.x0, src, R);
    else run_step<real, true, TRT, RN>(I, tl.x0, src, R);
}

// Workgroup -> contiguous run of tiles.  Workgroups are dealt round-robin to
// the 8 XCDs; renumbering them so each XCD gets a contiguous block of logical
// ids keeps vertically adjacent tiles (which share ring rows) in one L2.
__device__ inline void my_tiles(int ntiles, int& t0, int& t1)
{
    const int G = gridDim.x, b = blockIdx.x;
    const int xcd = b % 8, per = G / 8, rem = G % 8;
    const int L = xcd * per + (xcd < rem ? xcd : rem) + b / 8;
    t0 = (int)((long long)L * ntiles / G);
    t1 = (int)((long long)(L + 1) * ntiles / G);
}

// One step of every tile in the table, one node per work-item.
// VAR 0: every lattice of the launch uses BGK and the capillary term of Eq. 11;
// VAR 1: some lattice uses two relaxation times; VAR 2: some lattice uses the
// potential form of the capillary force (extra LDS, a second ring of phi).
// Separate kernels, so that the BGK-only kernel keeps its own register budget.
// RUNS: the table may also hold runs of TX * TY nodes (kTileRun entries; BGK
// or two relaxation times only); tile and run patches share the LDS.
template <typename real, int TX, int TY, int VAR, bool RUNS = false>
__global__ __launch_bounds__(TX* TY) void k_step(const Inst<real>* __restrict__ insts, const Tile* __restrict__ tiles,
                                                  int ntiles, int src)
{
    constexpr bool ANY_TRT = VAR >= 1;
    static_assert(!RUNS || VAR < 2, "runs: no potential form");
    using LDS = typename std::conditional<RUNS, StepLDS<real, TX, TY>, Patch<real, TX, TY>>::type;
    __shared__ LDS U;
    int t0, t1;
    my_tiles(ntiles, t0, t1);
    for (int t = t0; t < t1; ++t) {
        // the tile entry is the same for the whole workgroup: keep it scalar
        Tile tl = tiles[t];
        tl.inst = __builtin_amdgcn_readfirstlane(tl.inst);
        tl.x0 = __builtin_amdgcn_readfirstlane(tl.x0);
        tl.y0 = __builtin_amdgcn_readfirstlane(tl.y0);
        tl.flags = __builtin_amdgcn_readfirstlane(tl.flags);
        const Inst<real>& I = insts[tl.inst];
        Patch<real, TX, TY>* Sp;
        if constexpr (RUNS) Sp = &U.tile;
        else Sp = &U;
        Patch<real, TX, TY>& S = *Sp;
        if constexpr (VAR == 2) {
            __shared__ PotLDS<real, TX, TY> Q;
            if (I.collision == 0) tile_pot<real, TX, TY, false>(I, tl, src, S, Q);
            else tile_pot<real, TX, TY, true>(I, tl, src, S, Q);
        } else if (RUNS && (tl.flags & kTileRun)) {
            if constexpr (RUNS) {
                if (!ANY_TRT || I.collision == 0) run_any<real, false, TX * TY>(I, tl, src, U.run);
                else run_any<real, true, TX * TY>(I, tl, src, U.run);
            }
        } else {
            if (!ANY_TRT || I.collision == 0) tile_any<real, TX, TY, false>(I, tl, src, S);
            else tile_any<real, TX, TY, true>(I, tl, src, S);
        }
        if (t + 1 < t1) __syncthreads();
    }
}

template <typename real, typename out_t>
__device__ inline void put(void* p, long long i, real v)
{
    if (p) static_cast<out_t*>(p)[i] = static_cast<out_t>(v);
}

template <typename real, int TX, int TY>
__global__ __launch_bounds__(TX* TY) void k_fields(const Inst<real>* __restrict__ insts, const Tile* __restrict__ tiles,
                                                    int ntiles, int src, void* ophi, void* oux, void* ouy, void* oT,
                                                    void* op, int out_f32, int jprev_out)
{
    __shared__ Patch<real, TX, TY> S;
    __shared__ PotLDS<real, TX, TY> Q;
    int t0, t1;
    my_tiles(ntiles, t0, t1);
    for (int t = t0; t < t1; ++t) {
        const Tile tl = tiles[t];
        const Inst<real>& I = insts[tl.inst];
        real f[9], g[9], h[9];
        const bool inside = load_any(I, tl, src, S, f, g, h);
        if (I.force_form == 1) fill_mu<real, TX, TY>(I, src, S, Q, tl.x0, tl.y0);
        if (inside) {
            const int tid = threadIdx.x;
            const int gi = tl.x0 + tid % TX, gj = tl.y0 + tid / TX;
            constexpr int PX = Patch<real, TX, TY>::PX;
            const int c = (tid / TX + 1) * PX + (tid % TX + 1);
            const Macro<real> m = node_macros<real, GridNb<PX>, true>(I, S.phi, S.T, c, GridNb<PX>{}, g, Q.mu);
            if (jprev_out) {
                const long long own = (long long)gj * I.pitch + gi;
                const gptr<real> J = to_global(I.jprev);
                J[own] = m.phi * m.ux;
                J[I.plane + own] = m.phi * m.uy;
            } else {
                const long long o = (long long)gj * I.nx + gi;
                const double phi = (double)I.phi0 + (double)m.dphi;
                const double T = (double)I.T0 + (double)m.theta;
                if (out_f32) {
                    put<double, float>(ophi, o, phi);
                    put<real, float>(oux, o, m.ux);
                    put<real, float>(ouy, o, m.uy);
                    put<double, float>(oT, o, T);
                    put<real, float>(op, o, m.p);
                } else {
                    put<double, double>(ophi, o, phi);
                    put<real, double>(oux, o, m.ux);
                    put<real, double>(ouy, o, m.uy);
                    put<double, double>(oT, o, T);
                    put<real, double>(op, o, m.p);
                }
            }
        }
        if (t + 1 < t1) __syncthreads();
    }
}

// Equilibrium populations for given fields (p = 0): f_i = w_i phi (1 + 3 c_i.u),
// g_i = rho s_i(u), h_i = w_i T, stored as deviations.  Computed in FP64.
template <typename real>
__global__ void k_init(const Inst<real>* __restrict__ insts, const double* __restrict__ staged, double phi0,
                       double T0, double rho_a, double rho_b, int has_p, int shift, int src)
{
    const Inst<real>& I = insts[0];
    const long long n = (long long)I.nx * I.ny;
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    const int i = (int)(x % I.nx), j = (int)(x / I.nx);
    const double phi = staged[x], ux = staged[n + x], uy = staged[2 * n + x], T = staged[3 * n + x];
    const gptr<real> __restrict__ A = to_global(I.pop[src]);
    const long long idx = (long long)j * I.pitch + i;
    if (!shift) {
        const double p = has_p ? staged[4 * n + x] : 0.0;
        const double rho = rho_a + rho_b * phi;
        const double uu = ux * ux + uy * uy;
#pragma unroll
        for (int k = 0; k < 9; ++k) {
            const double w = wgt<double>(k);
            const double cu = cx(k) * ux + cy(k) * uy;
            A[pop_index(kF + k, idx)] = (real)(w * ((phi - phi0) + 3.0 * phi * cu));
            A[pop_index(kG + k, idx)] =
                (real)(3.0 * p * (w - (k == 0 ? 1.0 : 0.0)) + rho * w * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
            A[pop_index(kH + k, idx)] = (real)(w * (T - T0));
        }
        return;
    }
    // shift: add eq(new) - eq(current) to the populations, keeping their
    // non-equilibrium part; the current fields sit in staged planes 5..9
    const double phc = staged[5 * n + x], uxc = staged[6 * n + x], uyc = staged[7 * n + x];
    const double Tc = staged[8 * n + x], pc = staged[9 * n + x];
    const double p = has_p ? staged[4 * n + x] : pc;
    const double rho = rho_a + rho_b * phi, rhoc = rho_a + rho_b * phc;
    const double uu = ux * ux + uy * uy, uuc = uxc * uxc + uyc * uyc;
#pragma unroll
    for (int k = 0; k < 9; ++k) {
        const double w = wgt<double>(k);
        const double cu = cx(k) * ux + cy(k) * uy, cuc = cx(k) * uxc + cy(k) * uyc;
        const double df = w * ((phi - phc) + 3.0 * (phi * cu - phc * cuc));
        const double dg = 3.0 * (p - pc) * (w - (k == 0 ? 1.0 : 0.0)) +
                          w * (rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu) - rhoc * (3.0 * cuc + 4.5 * cuc * cuc - 1.5 * uuc));
        const double dh = w * (T - Tc);
        A[pop_index(kF + k, idx)] = (real)((double)A[pop_index(kF + k, idx)] + df);
        A[pop_index(kG + k, idx)] = (real)((double)A[pop_index(kG + k, idx)] + dg);
        A[pop_index(kH + k, idx)] = (real)((double)A[pop_index(kH + k, idx)] + dh);
    }
}

// Gathers device fields (FP32 or FP64, x fastest) into the FP64 staging layout
// k_init reads: [phi | ux | uy | T | p], n values each (p only if given).
template <typename in_t>
__global__ void k_stage(const in_t* __restrict__ phi, const in_t* __restrict__ ux, const in_t* __restrict__ uy,
                        const in_t* __restrict__ T, const in_t* __restrict__ p, long long n,
                        double* __restrict__ staged)
{
    const long long x = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (x >= n) return;
    staged[x] = (double)phi[x];
    staged[n + x] = (double)ux[x];
    staged[2 * n + x] = (double)uy[x];
    staged[3 * n + x] = (double)T[x];
    if (p) staged[4 * n + x] = (double)p[x];
}

hipError_t launch_stage(const void* phi, const void* ux, const void* uy, const void* T, const void* p, int in_f32,
                        long long n, double* staged, hipStream_t s)
{
    const dim3 grid((unsigned)((n + 255) / 256));
    if (in_f32)
        hipLaunchKernelGGL(k_stage<float>, grid, dim3(256), 0, s, static_cast<const float*>(phi),
                           static_cast<const float*>(ux), static_cast<const float*>(uy),
                           static_cast<const float*>(T), static_cast<const float*>(p), n, staged);
    else
        hipLaunchKernelGGL(k_stage<double>, grid, dim3(256), 0, s, static_cast<const double*>(phi),
                           static_cast<const double*>(ux), static_cast<const double*>(uy),
                           static_cast<const double*>(T), static_cast<const double*>(p), n, staged);
    return hipGetLastError();
}

// ---- FP64 diagnostics ----

__device__ inline double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ inline double wave_max(double v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
    return v;
}

template <typename real, int TX, int TY>
__global__ __launch_bounds__(TX* TY) void k_diag(const Inst<real>* __restrict__ insts, const Tile* __restrict__ tiles,
                                                  int ntiles, int src, DiagArgs a, double rcp_a, double rcp_b,
                                                  double* __restrict__ partials)
{
    __shared__ Patch<real, TX, TY> S;
    __shared__ PotLDS<real, TX, TY> Q;
    __shared__ double red[(TX * TY) / 64][D_COUNT];
    double acc[D_COUNT];
#pragma unroll
    for (int q = 0; q < D_COUNT; ++q) acc[q] = 0.0;
    int t0, t1;
    my_tiles(ntiles, t0, t1);
    for (int t = t0; t < t1; ++t) {
        const Tile tl = tiles[t];
        const Inst<real>& I = insts[tl.inst];
        real f[9], g[9], h[9];
        const bool inside = load_any(I, tl, src, S, f, g, h);
        if (I.force_form == 1) fill_mu<real, TX, TY>(I, src, S, Q, tl.x0, tl.y0);
        if (inside) {
            const int tid = threadIdx.x;
            const int gi = tl.x0 + tid % TX, gj = tl.y0 + tid / TX;
            constexpr int PX = Patch<real, TX, TY>::PX;
            const int c = (tid / TX + 1) * PX + (tid % TX + 1);
            const Macro<real> m = node_macros<real, GridNb<PX>, true>(I, S.phi, S.T, c, GridNb<PX>{}, g, Q.mu);
            const double phi = (double)I.phi0 + (double)m.dphi;
            const double T = (double)I.T0 + (double)m.theta;
            const double ux = m.ux, uy = m.uy, p = m.p;
            if (!isfinite(phi) || !isfinite(T) || !isfinite(ux) || !isfinite(uy) || !isfinite(p)) {
                acc[D_NONFIN] += 1.0;
            } else {
                acc[D_MASS] += phi;
                acc[D_VOL] += 0.5 * (1.0 - phi);
                acc[D_HEAT] += (rcp_a + rcp_b * phi) * T;
                acc[D_MAXU] = fmax(acc[D_MAXU], sqrt(ux * ux + uy * uy));
                if (phi < 0.0) {
                    acc[D_NNEG] += 1.0;
                    acc[D_SNEG] += phi;
                    acc[D_SUY] += phi * uy;
                    acc[D_SUX] += phi * ux;
                    acc[D_SX] += phi * gi;
                    acc[D_SY] += phi * gj;
                    if (a.n_bubbles > 0) {
                        int best = 0;
                        double bd = 0.0;
                        for (int b = 0; b < a.n_bubbles; ++b) {
                            const double dx = gi - a.bx[b], dy = gj - a.by[b];
                            const double d2 = dx * dx + dy * dy;
                            if (b == 0 || d2 < bd) { bd = d2; best = b; }
                        }
#pragma unroll
                        for (int b = 0; b < 4; ++b) {
                            if (b == best) {
                                acc[D_BUB + 5 * b + 0] += phi;
                                acc[D_BUB + 5 * b + 1] += phi * gi;
                                acc[D_BUB + 5 * b + 2] += phi * gj;
                                acc[D_BUB + 5 * b + 3] += phi * ux;
                                acc[D_BUB + 5 * b + 4] += phi * uy;
                            }
                        }
                    }
                }
            }
        }
        __syncthreads();
    }
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll
    for (int q = 0; q < D_COUNT; ++q) {
        const double v = q == D_MAXU ? wave_max(acc[q]) : wave_sum(acc[q]);
        if (lane == 0) red[wave][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < D_COUNT) {
        const int q = threadIdx.x;
        double v = red[0][q];
        for (int w = 1; w < (TX * TY) / 64; ++w) v = q == D_MAXU ? fmax(v, red[w][q]) : v + red[w][q];
        partials[(long long)blockIdx.x * D_COUNT + q] = v;
    }
}

__global__ __launch_bounds__(256) void k_diag_final(const double* __restrict__ partials, int nblocks,
                                                    double* __restrict__ result)
{
    __shared__ double red[4][D_COUNT];
    const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
    for (int q = 0; q < D_COUNT; ++q) {
        double v = 0.0;
        for (int b = threadIdx.x; b < nblocks; b += 256) {
            const double x = partials[(long long)b * D_COUNT + q];
            v = q == D_MAXU ? fmax(v, x) : v + x;
        }
        v = q == D_MAXU ? wave_max(v) : wave_sum(v);
        if (lane == 0) red[wave][q] = v;
    }
    __syncthreads();
    if (threadIdx.x < D_COUNT) {
        const int q = threadIdx.x;
        double v = red[0][q];
        for (int w = 1; w < 4; ++w) v = q == D_MAXU ? fmax(v, red[w][q]) : v + red[w][q];
        result[q] = v;
    }
}

// ---- plain copy (bandwidth and counter calibration) ----

__global__ __launch_bounds__(256) void k_copy(const float4* __restrict__ src, float4* __restrict__ dst, long long n)
{
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
        dst[i] = src[i];
}

hipError_t launch_copy(const void* src, void* dst, size_t bytes, hipStream_t s)
{
    const long long n = (long long)(bytes / sizeof(float4));
    long long blocks = (n + 255) / 256;
    if (blocks > 65536) blocks = 65536;
    if (blocks < 1) blocks = 1;
    hipLaunchKernelGGL(k_copy, dim3((unsigned)blocks), dim3(256), 0, s, static_cast<const float4*>(src),
                       static_cast<float4*>(dst), n);
    return hipGetLastError();
}

// ---- launchers ----

template <typename real, int TX, int TY, bool RUNS = false>
static hipError_t step_t(const void* insts, const Tile* tiles, int ntiles, int grid, int src, int variant,
                         hipStream_t s)
{
    const int G = grid > 0 ? grid : ntiles;
    const Inst<real>* ip = static_cast<const Inst<real>*>(insts);
    // a table for lattices with the potential form holds no runs
    if (variant == 2)
        hipLaunchKernelGGL((k_step<real, TX, TY, 2>), dim3(G), dim3(TX * TY), 0, s, ip, tiles, ntiles, src);
    else if (variant == 1)
        hipLaunchKernelGGL((k_step<real, TX, TY, 1, RUNS>), dim3(G), dim3(TX * TY), 0, s, ip, tiles, ntiles, src);
    else
        hipLaunchKernelGGL((k_step<real, TX, TY, 0, RUNS>), dim3(G), dim3(TX * TY), 0, s, ip, tiles, ntiles, src);
    return hipGetLastError();
}

template <typename real, int TX, int TY>
static hipError_t fields_t(const void* insts, const Tile* tiles, int ntiles, int src, void* phi, void* ux, void* uy,
                           void* T, void* p, int out_f32, int jprev_out, hipStream_t s)
{
    hipLaunchKernelGGL((k_fields<real, TX, TY>), dim3(ntiles), dim3(TX * TY), 0, s,
                       static_cast<const Inst<real>*>(insts), tiles, ntiles, src, phi, ux, uy, T, p, out_f32,
                       jprev_out);
    return hipGetLastError();
}

template <typename real, int TX, int TY>
static hipError_t diag_t(const void* insts, const Tile* tiles, int ntiles, int src, const DiagArgs& a,
                         double rcp_a, double rcp_b, double* partials, double* result, hipStream_t s)
{
    hipLaunchKernelGGL((k_diag<real, TX, TY>), dim3(ntiles), dim3(TX * TY), 0, s,
                       static_cast<const Inst<real>*>(insts), tiles, ntiles, src, a, rcp_a, rcp_b, partials);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(256), 0, s, partials, ntiles, result);
    return hipGetLastError();
}

// Tile id -> (TX, TY), in the order of kTileTX and kTileTY (the field and
// diagnostics kernels take grid_tile(id)).
#define LBM_TILE_SWITCH(TILE, CALL)                  \
    switch (TILE) {                                  \
    case 0: return CALL(64, 4);                      \
    case 1: return CALL(128, 2);                     \
    case 2: return CALL(32, 8);                      \
    case 3: return CALL(64, 8);                      \
    case 4: return CALL(256, 1);                     \
    case 5: return CALL(128, 4);                     \
    default: return hipErrorInvalidValue;            \
    }
static_assert(kTileCount == 8 && kTileTX[6] == 128 && kTileTY[6] == 4 && grid_tile(6) == 5 && kTileTX[7] == 64 &&
                  kTileTY[7] == 4 && grid_tile(7) == 0,
              "runs of 512 nodes take the 128 x 4 kernel, runs of 256 the 64 x 4 kernel");

hipError_t launch_step(int prec, int tile, const void* insts, const Tile* tiles, int ntiles, int grid, int src,
                       int variant, hipStream_t s)
{
#define STEP64(a, b) step_t<double, a, b>(insts, tiles, ntiles, grid, src, variant, s)
#define STEP32(a, b) step_t<float, a, b>(insts, tiles, ntiles, grid, src, variant, s)
    if (tile == 6)
        return prec == 0 ? step_t<double, 128, 4, true>(insts, tiles, ntiles, grid, src, variant, s)
                         : step_t<float, 128, 4, true>(insts, tiles, ntiles, grid, src, variant, s);
    if (tile == 7)
        return prec == 0 ? step_t<double, 64, 4, true>(insts, tiles, ntiles, grid, src, variant, s)
                         : step_t<float, 64, 4, true>(insts, tiles, ntiles, grid, src, variant, s);
    if (prec == 0) { LBM_TILE_SWITCH(tile, STEP64) }
    LBM_TILE_SWITCH(tile, STEP32)
#undef STEP64
#undef STEP32
}

template <typename real, int TX, int TY, bool RUNS = false>
static hipError_t occ_t(int* blocks, int variant)
{
    if (variant == 2) return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_step<real, TX, TY, 2>, TX * TY, 0);
    if (variant == 1)
        return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_step<real, TX, TY, 1, RUNS>, TX * TY, 0);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks, k_step<real, TX, TY, 0, RUNS>, TX * TY, 0);
}

hipError_t step_occupancy(int prec, int tile, int variant, int* blocks_per_cu)
{
#define O64(a, b) occ_t<double, a, b>(blocks_per_cu, variant)
#define O32(a, b) occ_t<float, a, b>(blocks_per_cu, variant)
    if (tile == 6)
        return prec == 0 ? occ_t<double, 128, 4, true>(blocks_per_cu, variant)
                         : occ_t<float, 128, 4, true>(blocks_per_cu, variant);
    if (tile == 7)
        return prec == 0 ? occ_t<double, 64, 4, true>(blocks_per_cu, variant)
                         : occ_t<float, 64, 4, true>(blocks_per_cu, variant);
    if (prec == 0) { LBM_TILE_SWITCH(tile, O64) }
    LBM_TILE_SWITCH(tile, O32)
#undef O64
#undef O32
}

hipError_t launch_fields(int prec, int tile, const void* insts, const Tile* tiles, int ntiles, int src, void* phi,
                         void* ux, void* uy, void* T, void* p, int out_f32, int jprev_out, hipStream_t s)
{
#define F64(a, b) fields_t<double, a, b>(insts, tiles, ntiles, src, phi, ux, uy, T, p, out_f32, jprev_out, s)
#define F32(a, b) fields_t<float, a, b>(insts, tiles, ntiles, src, phi, ux, uy, T, p, out_f32, jprev_out, s)
    if (prec == 0) { LBM_TILE_SWITCH(tile, F64) }
    LBM_TILE_SWITCH(tile, F32)
#undef F64
#undef F32
}

hipError_t launch_init(int prec, const void* inst_dev, long long n_nodes, const double* staged, const InitArgs& a,
                       int src, hipStream_t s)
{
    const dim3 grid((unsigned)((n_nodes + 255) / 256));
    if (prec == 0)
        hipLaunchKernelGGL(k_init<double>, grid, dim3(256), 0, s, static_cast<const Inst<double>*>(inst_dev), staged,
                           a.phi0, a.T0, a.rho_a, a.rho_b, a.has_p, a.shift, src);
    else
        hipLaunchKernelGGL(k_init<float>, grid, dim3(256), 0, s, static_cast<const Inst<float>*>(inst_dev), staged,
                           a.phi0, a.T0, a.rho_a, a.rho_b, a.has_p, a.shift, src);
    return hipGetLastError();
}

hipError_t launch_diag(int prec, int tile, const void* insts, const Tile* tiles, int ntiles, int src,
                       const DiagArgs& a, double* partials, double* result, hipStream_t s)
{
#define D64(x, y) diag_t<double, x, y>(insts, tiles, ntiles, src, a, a.rcp_a, a.rcp_b, partials, result, s)
#define D32(x, y) diag_t<float, x, y>(insts, tiles, ntiles, src, a, a.rcp_a, a.rcp_b, partials, result, s)
    if (prec == 0) { LBM_TILE_SWITCH(tile, D64) }
    LBM_TILE_SWITCH(tile, D32)
#undef D64
#undef D32
}

}  // namespace lbm
