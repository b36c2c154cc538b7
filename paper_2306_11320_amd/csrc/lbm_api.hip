// Host side of the C ABI declared in include/lbm.h: parameter validation,
// workspace carving, tile tables, HIP graph capture of step sequences,
// diagnostics and state transfer.  All lattice arithmetic runs in the kernels
// of lbm_kernels.hip.
#include "lbm.h"
#include "lbm_internal.hpp"

#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail(int code, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(expr)                                                                       \
    do {                                                                                    \
        hipError_t e_ = (expr);                                                             \
        if (e_ != hipSuccess) return fail(LBM_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr size_t kAlign = 256;
// Nodes per row boundary: FP32 rows start on 64-byte boundaries of a
// population run, FP64 rows are packed with no gap; rows of lattices that runs
// can step are packed in both (see make_layout).
int row_align(size_t rsz) { return rsz == 8 ? 1 : 16; }
size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

constexpr double W9[9] = {4.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0, 1.0 / 9.0,
                          1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};

struct Layout {
    int nx, ny, pitch;
    long long plane;        // elements per plane
    size_t pop_off[2];      // byte offsets of time levels A and B
    size_t jprev_off;
    size_t twall_off;       // byte offset of the wall-temperature tables
    int tw_stride;          // entries per side
    int tile_off[lbm::kTileCount], tile_cnt[lbm::kTileCount];
};

size_t real_size(uint32_t prec) { return prec == LBM_FP64 ? sizeof(double) : sizeof(float); }

int validate(const lbm_params& p)
{
    if (p.abi_version != LBM_ABI_VERSION) return fail(LBM_EINVAL, "abi_version %u != %u", p.abi_version, LBM_ABI_VERSION);
    if (p.nx < 3 || p.ny < 3) return fail(LBM_EINVAL, "lattice %ux%u smaller than 3x3", p.nx, p.ny);
    if (p.nx > (uint32_t)INT_MAX || p.ny > (uint32_t)INT_MAX)
        return fail(LBM_EINVAL, "lattice %ux%u: sizes must fit a signed 32-bit integer", p.nx, p.ny);
    // node offsets within a level are 32-bit byte offsets in the kernels
    const uint64_t word = p.precision == LBM_FP64 ? 8 : 4, row = (uint64_t)row_align(word);
    if (((uint64_t)(p.nx + row - 1) / row * row * p.ny + lbm::kBlock - 1) / lbm::kBlock * lbm::kBlock * lbm::kPlanes *
            word >= (1ull << 32))
        return fail(LBM_EINVAL, "lattice too large (%ux%u): a time level must stay below 4 GiB", p.nx, p.ny);
    if (p.precision != LBM_FP64 && p.precision != LBM_FP32_DEV) return fail(LBM_EINVAL, "unknown precision %u", p.precision);
    for (int s = 0; s < 4; ++s)
        if (p.bc[s] > LBM_BC_OUTLET) return fail(LBM_EINVAL, "unknown boundary kind %u on side %d", p.bc[s], s);
    if ((p.bc[0] == LBM_BC_PERIODIC) != (p.bc[1] == LBM_BC_PERIODIC))
        return fail(LBM_EINVAL, "x sides: periodic paired with a non-periodic side");
    if ((p.bc[2] == LBM_BC_PERIODIC) != (p.bc[3] == LBM_BC_PERIODIC))
        return fail(LBM_EINVAL, "y sides: periodic paired with a non-periodic side");
    if (p.grad_mode > 1) return fail(LBM_EINVAL, "grad_mode must be 0 or 1");
    if (p.collision != LBM_BGK && p.collision != LBM_TRT) return fail(LBM_EINVAL, "unknown collision %u", p.collision);
    if (p.force_form != LBM_FORCE_EQ11 && p.force_form != LBM_FORCE_POTENTIAL)
        return fail(LBM_EINVAL, "unknown force_form %u", p.force_form);
    if (p.collision == LBM_TRT && !(p.trt_magic > 0)) return fail(LBM_EINVAL, "trt_magic must be positive");
    if (p.n_bubbles > 4) return fail(LBM_EINVAL, "at most 4 tracked regions");
    if (!(p.rho_l > 0 && p.rho_h > 0)) return fail(LBM_EINVAL, "densities must be positive");
    if (!(p.mu_l > 0 && p.mu_h > 0)) return fail(LBM_EINVAL, "viscosities must be positive (tau_g > 1/2)");
    if (!(p.lambda_l > 0 && p.lambda_h > 0)) return fail(LBM_EINVAL, "conductivities must be positive (tau_h > 1/2)");
    if (!(p.rhocp_l > 0 && p.rhocp_h > 0)) return fail(LBM_EINVAL, "heat capacitances must be positive");
    if (!(p.mobility > 0)) return fail(LBM_EINVAL, "mobility must be positive (tau_phi > 1/2)");
    if (!(p.W > 0)) return fail(LBM_EINVAL, "interface width must be positive");
    // The destination blend of Eq. 28, h_i <- [h*_i + (rho c_p - 1) h_i] / rho c_p,
    // is a convex combination only for rho c_p >= 1: accepted, with a warning
    // left in the thread's message text.
    if (p.rhocp_l < 1.0 || p.rhocp_h < 1.0)
        (void)fail(LBM_OK, "warning: heat capacitance below 1 (%g, %g): the blend of Eq. 28 is not convex",
                   p.rhocp_l, p.rhocp_h);
    return LBM_OK;
}

// Step kernel of a set of lattices: 0 BGK only; 1 some lattice relaxes with
// two relaxation times; 2 some lattice uses the potential form of the
// capillary force.
int step_variant(const lbm_params* ps, int n)
{
    int v = 0;
    for (int k = 0; k < n; ++k) {
        if (ps[k].collision == LBM_TRT && v < 1) v = 1;
        if (ps[k].force_form == LBM_FORCE_POTENTIAL) v = 2;
    }
    return v;
}

// Whether the run tile ids step the lattice in runs (else in its tiles).
bool runs_for(const lbm_params& p, int variant)
{
    return variant < 2 && p.bc[0] == LBM_BC_PERIODIC && p.nx >= (uint32_t)lbm::kRunMinNx &&
           p.nx <= (uint32_t)lbm::kRunMaxNx;
}

Layout make_layout(const lbm_params& p, size_t rsz, int variant, size_t& cursor)
{
    Layout L{};
    L.nx = (int)p.nx;
    L.ny = (int)p.ny;
    // Rows are not padded to whole blocks: a row whose width is not a multiple
    // of the block shares its last block with the next row, so no slot that
    // no node owns is moved (measured on the batched sweep, FP64: 1.15 ->
    // 1.07 ms per step).  In FP32, tiles on rows whose starts are not 8-byte
    // aligned were measured up to 10% slower; there rows start on 64-byte
    // boundaries (at most 15 slots between rows, written as zeros by the
    // step), except in lattices that runs can step: packed rows keep a run's
    // nodes contiguous in memory, so every wavefront of a run reads whole
    // aligned runs of 64 values (width 221: 51.5 -> 45.5 ps per node).
    L.pitch = runs_for(p, variant) ? (int)p.nx : (int)align_up(p.nx, (size_t)row_align(rsz));
    L.plane = (long long)align_up(align_up((size_t)L.pitch * p.ny, lbm::kBlock), kAlign / rsz);
    const size_t level = (size_t)lbm::kPlanes * L.plane * rsz;
    L.pop_off[0] = cursor;
    cursor = align_up(cursor + level, kAlign);
    L.pop_off[1] = cursor;
    cursor = align_up(cursor + level, kAlign);
    L.jprev_off = cursor;
    cursor = align_up(cursor + 2 * (size_t)L.plane * rsz, kAlign);
    // wall temperatures at s = -kTwPad/2 ... max(nx, ny) + kTwPad/2 - 1/2 in
    // steps of 1/2, for each of the four sides
    L.tw_stride = 2 * (L.nx > L.ny ? L.nx : L.ny) + 2 * lbm::kTwPad;
    L.twall_off = cursor;
    cursor = align_up(cursor + 4 * (size_t)L.tw_stride * rsz, kAlign);
    return L;
}

int tiles_of(const Layout& L, const lbm_params& p, int variant, int t)
{
    const int rn = lbm::run_nodes(t);
    if (rn && runs_for(p, variant)) return (int)(((long long)L.nx * L.ny + rn - 1) / rn);
    const int tx = lbm::kTileTX[t], ty = lbm::kTileTY[t];
    return ((L.nx + tx - 1) / tx) * ((L.ny + ty - 1) / ty);
}

template <typename real>
lbm::Inst<real> make_inst(const lbm_params& p, const Layout& L, char* ws)
{
    lbm::Inst<real> I{};
    I.pop[0] = reinterpret_cast<real*>(ws + L.pop_off[0]);
    I.pop[1] = reinterpret_cast<real*>(ws + L.pop_off[1]);
    I.jprev = reinterpret_cast<real*>(ws + L.jprev_off);
    for (int l = 0; l < 2; ++l)
        for (int q = 0; q < 27; ++q) I.qbase[l][q] = I.pop[l] + lbm::pop_index(q, 0);
    I.jbase[0] = I.jprev;
    I.jbase[1] = I.jprev + L.plane;
    I.nx = L.nx;
    I.ny = L.ny;
    I.pitch = L.pitch;
    I.plane = L.plane;
    I.grad_mode = (int)p.grad_mode;
    I.collision = (int)p.collision;
    I.force_form = (int)p.force_form;
    I.trt_magic = (real)p.trt_magic;
    for (int s = 0; s < 4; ++s) I.bc[s] = (int)p.bc[s];
    const double phi0 = p.phi0_dev, T0 = p.T0_dev;
    I.phi0 = (real)phi0;
    I.T0 = (real)T0;
    // xi(phi) = xi_l (1 - phi)/2 + xi_h (1 + phi)/2 = xi_a + xi_b phi
    I.rho_a = (real)(0.5 * (p.rho_l + p.rho_h));
    I.rho_b = (real)(0.5 * (p.rho_h - p.rho_l));
    I.mu_a = (real)(0.5 * (p.mu_l + p.mu_h));
    I.mu_b = (real)(0.5 * (p.mu_h - p.mu_l));
    I.lam_a = (real)(0.5 * (p.lambda_l + p.lambda_h));
    I.lam_b = (real)(0.5 * (p.lambda_h - p.lambda_l));
    I.rcp_a = (real)(0.5 * (p.rhocp_l + p.rhocp_h));
    I.rcp_b = (real)(0.5 * (p.rhocp_h - p.rhocp_l));
    I.sigma_ref = (real)p.sigma_ref;
    I.sigma_T = (real)p.sigma_T;
    I.sigma_TT = (real)p.sigma_TT;
    I.dTref = (real)(T0 - p.T_ref);
    I.W2 = (real)(p.W * p.W);
    I.pref = (real)(3.0 * std::sqrt(2.0) * p.W / 4.0);
    I.inv_W2 = (real)(1.0 / (p.W * p.W));
    I.inv_s2W = (real)(1.0 / (std::sqrt(2.0) * p.W));
    const double tau_phi = 0.5 + 3.0 * p.mobility;  // M = c_s^2 (tau_phi - 1/2)
    I.inv_tau_phi = (real)(1.0 / tau_phi);
    I.fac_phi = (real)(1.0 - 0.5 / tau_phi);
    I.Gx = (real)p.Gx;
    I.Gy = (real)p.Gy;
    I.twall = reinterpret_cast<const real*>(ws + L.twall_off);
    I.tw_stride = L.tw_stride;
    I.u_in = (real)p.u_in_mean;
    I.phi_in_d = (real)(p.phi_in - phi0);
    I.T_in_d = (real)(p.T_in - T0);
    return I;
}

// Wall temperatures relative to T0 at s = (j - kTwPad) / 2 along each side,
// T_w(s) = Tw_mean + Tw_amp cos(Tw_k s) + Tw_slope s, for the boundary rules
// of the step kernel; copied into the lattice's table (the stream is
// synchronized before the host copy is freed).
template <typename real>
hipError_t put_wall_table(const lbm_params& p, const Layout& L, char* ws, hipStream_t s)
{
    std::vector<real> t(4 * (size_t)L.tw_stride);
    for (int side = 0; side < 4; ++side)
        for (int j = 0; j < L.tw_stride; ++j) {
            const double x = 0.5 * (j - lbm::kTwPad);
            const double Tw = p.Tw_mean[side] + p.Tw_amp[side] * std::cos(p.Tw_k[side] * x) + p.Tw_slope[side] * x;
            t[(size_t)side * L.tw_stride + j] = (real)(Tw - p.T0_dev);
        }
    hipError_t e = hipMemcpyAsync(ws + L.twall_off, t.data(), t.size() * sizeof(real), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e;
}

uint64_t params_hash(const std::vector<lbm_params>& ps)
{
    uint64_t h = 1469598103934665603ull;  // FNV-1a
    for (const auto& p : ps) {
        const unsigned char* b = reinterpret_cast<const unsigned char*>(&p);
        for (size_t i = 0; i < sizeof(p); ++i) {
            h ^= b[i];
            h *= 1099511628211ull;
        }
    }
    return h;
}

}  // namespace

struct lbm_ctx {
    uint32_t prec = 0;
    int n = 0;
    int tile = 0;
    int graph_steps = 64;
    int grid = 0;
    // step kernel: 0 BGK only; 1 some lattice relaxes with two relaxation
    // times; 2 some lattice uses the potential form of the capillary force
    int variant = 0;
    // some lattice is stepped in runs by the run tile ids (else those ids
    // repeat the tiles of their TX x TY shape)
    bool has_runs = false;
    hipStream_t stream = nullptr;
    char* ws = nullptr;
    size_t ws_bytes = 0;
    std::vector<lbm_params> params;
    std::vector<Layout> lay;
    std::vector<char> h_insts;  // host copy of the device Inst array
    void* d_insts = nullptr;
    lbm::Tile* d_tiles[lbm::kTileCount] = {};
    int ntiles[lbm::kTileCount] = {};
    double* d_partials = nullptr;
    double* d_result = nullptr;
    int64_t step = 0;
    hipGraphExec_t gexec = nullptr;
    int gexec_steps = 0;
    std::vector<double> bx, by;  // per instance, 4 tracked centroids
};

namespace {

size_t inst_size(uint32_t prec) { return prec == LBM_FP64 ? sizeof(lbm::Inst<double>) : sizeof(lbm::Inst<float>); }

// Carves the workspace; fills layouts and the offsets of the shared tables.
size_t plan(const lbm_params* ps, int n, std::vector<Layout>* lay, size_t* off_insts, size_t off_tiles[],
            size_t* off_partials, size_t* off_result)
{
    const uint32_t prec = ps[0].precision;
    const size_t rsz = real_size(prec);
    size_t cursor = 0;
    std::vector<Layout> L;
    int tot[lbm::kTileCount] = {};
    const int variant = step_variant(ps, n);
    for (int k = 0; k < n; ++k) {
        Layout l = make_layout(ps[k], rsz, variant, cursor);
        for (int t = 0; t < lbm::kTileCount; ++t) {
            l.tile_off[t] = tot[t];
            l.tile_cnt[t] = tiles_of(l, ps[k], variant, t);
            tot[t] += l.tile_cnt[t];
        }
        L.push_back(l);
    }
    *off_insts = cursor;
    cursor = align_up(cursor + (size_t)n * inst_size(prec), kAlign);
    int maxt = 1;
    for (int t = 0; t < lbm::kTileCount; ++t) {
        off_tiles[t] = cursor;
        cursor = align_up(cursor + (size_t)tot[t] * sizeof(lbm::Tile), kAlign);
        if (tot[t] > maxt) maxt = tot[t];
    }
    *off_partials = cursor;
    cursor = align_up(cursor + (size_t)maxt * lbm::D_COUNT * sizeof(double), kAlign);
    *off_result = cursor;
    cursor = align_up(cursor + lbm::D_COUNT * sizeof(double), kAlign);
    if (lay) *lay = L;
    return cursor;
}

void drop_graph(lbm_ctx* c)
{
    if (c->gexec) {
        (void)hipGraphExecDestroy(c->gexec);
        c->gexec = nullptr;
        c->gexec_steps = 0;
    }
}

int launch_one(lbm_ctx* c, int src)
{
    HIP_TRY(lbm::launch_step((int)c->prec, c->tile, c->d_insts, c->d_tiles[c->tile], c->ntiles[c->tile], c->grid, src,
                             c->variant, c->stream));
    return LBM_OK;
}

int capture(lbm_ctx* c)
{
    drop_graph(c);
    hipGraph_t g = nullptr;
    HIP_TRY(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    int rc = LBM_OK;
    for (int s = 0; s < c->graph_steps && rc == LBM_OK; ++s) rc = launch_one(c, s & 1);
    hipError_t e = hipStreamEndCapture(c->stream, &g);
    if (rc != LBM_OK) {
        if (g) (void)hipGraphDestroy(g);
        return rc;
    }
    if (e != hipSuccess) return fail(LBM_EHIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&c->gexec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return fail(LBM_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(e));
    c->gexec_steps = c->graph_steps;
    return LBM_OK;
}

int init_common(int n, const lbm_params* ps, const double* const* phi0, const double* const* ux0,
                const double* const* uy0, const double* const* T0, void* d_ws, size_t ws_bytes, void* stream,
                lbm_ctx** out)
{
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    *out = nullptr;
    if (n < 1 || !ps || !phi0 || !ux0 || !uy0 || !T0 || !d_ws) return fail(LBM_EINVAL, "NULL argument or n < 1");
    if (reinterpret_cast<uintptr_t>(d_ws) % kAlign) return fail(LBM_EINVAL, "workspace not 256-byte aligned");
    for (int k = 0; k < n; ++k) {
        int rc = validate(ps[k]);
        if (rc) return rc;
        if (ps[k].precision != ps[0].precision) return fail(LBM_EINVAL, "lattice %d: precision differs", k);
        if (!phi0[k] || !ux0[k] || !uy0[k] || !T0[k]) return fail(LBM_EINVAL, "lattice %d: NULL field", k);
    }
    std::vector<Layout> lay;
    size_t off_insts, off_tiles[lbm::kTileCount], off_part, off_res;
    const size_t need = plan(ps, n, &lay, &off_insts, off_tiles, &off_part, &off_res);
    if (ws_bytes < need) return fail(LBM_ENOSPACE, "workspace %zu bytes < %zu needed", ws_bytes, need);

    lbm_ctx* c = new (std::nothrow) lbm_ctx();
    if (!c) return fail(LBM_EINVAL, "out of host memory");
    c->prec = ps[0].precision;
    c->n = n;
    // default tile: 64 x 4 (FP64: measured fastest for single lattices; FP32:
    // see below once the tile tables exist)
    c->tile = 0;
    c->stream = static_cast<hipStream_t>(stream);
    c->ws = static_cast<char*>(d_ws);
    c->ws_bytes = ws_bytes;
    c->params.assign(ps, ps + n);
    c->variant = step_variant(ps, n);
    for (int k = 0; k < n; ++k) c->has_runs = c->has_runs || runs_for(ps[k], c->variant);
    c->lay = lay;
    c->grid = n > 1 ? -1 : 0;  // batched: persistent grid sized at the first step
    c->d_insts = c->ws + off_insts;
    c->d_partials = reinterpret_cast<double*>(c->ws + off_part);
    c->d_result = reinterpret_cast<double*>(c->ws + off_res);
    c->bx.assign(4 * (size_t)n, 0.0);
    c->by.assign(4 * (size_t)n, 0.0);
    const size_t isz = inst_size(c->prec);
    c->h_insts.resize((size_t)n * isz);
    for (int k = 0; k < n; ++k) {
        if (c->prec == LBM_FP64) {
            auto I = make_inst<double>(ps[k], lay[k], c->ws);
            std::memcpy(c->h_insts.data() + k * isz, &I, isz);
        } else {
            auto I = make_inst<float>(ps[k], lay[k], c->ws);
            std::memcpy(c->h_insts.data() + k * isz, &I, isz);
        }
        for (int b = 0; b < 4; ++b) {
            c->bx[4 * k + b] = ps[k].bubble_x[b];
            c->by[4 * k + b] = ps[k].bubble_y[b];
        }
    }
    auto bail = [&](int rc) {
        delete c;
        return rc;
    };
    hipError_t e = hipMemcpyAsync(c->d_insts, c->h_insts.data(), c->h_insts.size(), hipMemcpyHostToDevice, c->stream);
    if (e != hipSuccess) return bail(fail(LBM_EHIP, "copy of lattice constants: %s", hipGetErrorString(e)));
    for (int k = 0; k < n; ++k) {
        e = c->prec == LBM_FP64 ? put_wall_table<double>(ps[k], lay[k], c->ws, c->stream)
                                : put_wall_table<float>(ps[k], lay[k], c->ws, c->stream);
        if (e != hipSuccess) return bail(fail(LBM_EHIP, "copy of wall temperatures: %s", hipGetErrorString(e)));
    }
    // tile tables for every compiled shape, ordered by lattice then row-major
    // tiles (or runs in node order)
    for (int t = 0; t < lbm::kTileCount; ++t) {
        std::vector<lbm::Tile> tl;
        for (int k = 0; k < n; ++k) {
            const int tx = lbm::kTileTX[t], ty = lbm::kTileTY[t];
            const int nx = lay[k].nx, ny = lay[k].ny;
            const int rn = lbm::run_nodes(t);
            if (rn && runs_for(ps[k], c->variant)) {
                const long long nn = (long long)nx * ny;
                for (long long n0 = 0; n0 < nn; n0 += rn) {
                    const long long last = (n0 + rn < nn ? n0 + rn : nn) - 1;
                    // interior: no node of the first or last row
                    const bool inner = n0 / nx >= 1 && last / nx <= ny - 2;
                    tl.push_back(lbm::Tile{k, (int)n0, 0, lbm::kTileRun | (inner ? lbm::kTileInterior : 0)});
                }
                continue;
            }
            const bool px = ps[k].bc[0] == LBM_BC_PERIODIC, py = ps[k].bc[2] == LBM_BC_PERIODIC;
            for (int y = 0; y < ny; y += ty)
                for (int x = 0; x < nx; x += tx) {
                    const bool whole = x + tx <= nx && y + ty <= ny;
                    // wrap-only: in a periodic direction one wrap must reach
                    // every point of the tile and its ring (tile no longer
                    // than the lattice)
                    const bool inx = px ? (nx >= 3 && tx <= nx) : (x >= 1 && x + tx <= nx - 1);
                    const bool iny = py ? (ny >= 3 && ty <= ny) : (y >= 1 && y + ty <= ny - 1);
                    tl.push_back(lbm::Tile{k, x, y, (inx && iny ? lbm::kTileInterior : 0) | (whole ? lbm::kTileWhole : 0)});
                }
        }
        c->d_tiles[t] = reinterpret_cast<lbm::Tile*>(c->ws + off_tiles[t]);
        c->ntiles[t] = (int)tl.size();
        e = hipMemcpyAsync(c->d_tiles[t], tl.data(), tl.size() * sizeof(lbm::Tile), hipMemcpyHostToDevice, c->stream);
        if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return bail(fail(LBM_EHIP, "copy of tile table: %s", hipGetErrorString(e)));
    }
    // FP32: 64 x 8 when one round of resident workgroups covers every tile
    // (fewer ring reloads; 256 x 1024 lattice +1.8%), else 64 x 4 (later rounds
    // overlap earlier ones; 512 x 2048 lattice +2.3%)
    if (c->prec == LBM_FP32_DEV) {
        int dev = 0, cus = 0, per_cu = 0;
        if (hipGetDevice(&dev) == hipSuccess &&
            hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
            lbm::step_occupancy((int)c->prec, 3, c->variant, &per_cu) == hipSuccess && per_cu > 0 && cus > 0)
            c->tile = c->ntiles[3] <= per_cu * cus ? 3 : 0;
        else
            c->tile = 3;
    }
    // equilibrium populations: fields are staged in the lattice's level B
    for (int k = 0; k < n; ++k) {
        const size_t nn = (size_t)lay[k].nx * lay[k].ny;
        double* staged = reinterpret_cast<double*>(c->ws + lay[k].pop_off[1]);
        const double* src[4] = {phi0[k], ux0[k], uy0[k], T0[k]};
        for (int q = 0; q < 4; ++q) {
            e = hipMemcpyAsync(staged + q * nn, src[q], nn * sizeof(double), hipMemcpyHostToDevice, c->stream);
            if (e != hipSuccess) return bail(fail(LBM_EHIP, "copy of initial fields: %s", hipGetErrorString(e)));
        }
        lbm::InitArgs ia{ps[k].phi0_dev, ps[k].T0_dev, 0.5 * (ps[k].rho_l + ps[k].rho_h),
                         0.5 * (ps[k].rho_h - ps[k].rho_l), 0, 0};
        e = lbm::launch_init((int)c->prec, static_cast<char*>(c->d_insts) + k * isz, (long long)nn, staged, ia, 0,
                             c->stream);
        if (e != hipSuccess) return bail(fail(LBM_EHIP, "init kernel: %s", hipGetErrorString(e)));
        // the staging must be consumed before the next lattice reuses memory
        e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) return bail(fail(LBM_EHIP, "init: %s", hipGetErrorString(e)));
    }
    // (phi u) of the previous level := (phi u) now, so the first time derivative is zero
    const int ft = lbm::grid_tile(c->tile);
    e = lbm::launch_fields((int)c->prec, ft, c->d_insts, c->d_tiles[ft], c->ntiles[ft], 0, nullptr,
                           nullptr, nullptr, nullptr, nullptr, 0, 1, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return bail(fail(LBM_EHIP, "initial (phi u): %s", hipGetErrorString(e)));
    *out = c;
    return LBM_OK;
}

int check_instance(const lbm_ctx* c, int k)
{
    if (!c) return fail(LBM_EINVAL, "context is NULL");
    if (k < 0 || k >= c->n) return fail(LBM_EINVAL, "instance %d out of range [0, %d)", k, c->n);
    return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm_workspace_bytes(const lbm_params* p) { return lbm_workspace_bytes_batch(p, 1); }

size_t lbm_workspace_bytes_batch(const lbm_params* p, int n)
{
    if (!p || n < 1) return 0;
    for (int k = 0; k < n; ++k)
        if (validate(p[k]) != LBM_OK) return 0;
    size_t a, b[lbm::kTileCount], d, e;
    return plan(p, n, nullptr, &a, b, &d, &e);
}

int lbm_init(const lbm_params* p, const double* phi0, const double* ux0, const double* uy0, const double* T0,
             void* d_workspace, size_t ws_bytes, void* hip_stream, lbm_ctx** out)
{
    return init_common(1, p, &phi0, &ux0, &uy0, &T0, d_workspace, ws_bytes, hip_stream, out);
}

int lbm_init_batch(int n, const lbm_params* params, const double* const* phi0, const double* const* ux0,
                   const double* const* uy0, const double* const* T0, void* d_workspace, size_t ws_bytes,
                   void* hip_stream, lbm_ctx** out)
{
    return init_common(n, params, phi0, ux0, uy0, T0, d_workspace, ws_bytes, hip_stream, out);
}

int lbm_instances(const lbm_ctx* c) { return c ? c->n : 0; }

int lbm_step(lbm_ctx* c, int64_t n)
{
    if (!c) return fail(LBM_EINVAL, "context is NULL");
    if (n < 0) return fail(LBM_EINVAL, "negative step count");
    if (c->grid < 0) {
        int dev = 0, cus = 0;
        HIP_TRY(hipGetDevice(&dev));
        HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        c->grid = 8 * (cus > 0 ? cus : 256);
        if (c->grid > c->ntiles[c->tile]) c->grid = c->ntiles[c->tile];
    }
    while (n > 0) {
        if (c->graph_steps > 0 && (c->step & 1) == 0 && n >= c->graph_steps) {
            if (!c->gexec) {
                int rc = capture(c);
                if (rc) return rc;
            }
            HIP_TRY(hipGraphLaunch(c->gexec, c->stream));
            c->step += c->gexec_steps;
            n -= c->gexec_steps;
        } else {
            int rc = launch_one(c, (int)(c->step & 1));
            if (rc) return rc;
            c->step += 1;
            n -= 1;
        }
    }
    return LBM_OK;
}

int lbm_fields_instance(lbm_ctx* c, int instance, void* d_phi, void* d_ux, void* d_uy, void* d_T, void* d_p,
                        int out_dtype)
{
    int rc = check_instance(c, instance);
    if (rc) return rc;
    if (out_dtype != LBM_OUT_F64 && out_dtype != LBM_OUT_F32) return fail(LBM_EINVAL, "unknown output dtype");
    const Layout& L = c->lay[instance];
    const int ft = lbm::grid_tile(c->tile);
    HIP_TRY(lbm::launch_fields((int)c->prec, ft, c->d_insts, c->d_tiles[ft] + L.tile_off[ft],
                               L.tile_cnt[ft], (int)(c->step & 1), d_phi, d_ux, d_uy, d_T, d_p,
                               out_dtype == LBM_OUT_F32, 0, c->stream));
    return LBM_OK;
}

int lbm_reinit_fields(lbm_ctx* c, int instance, const void* d_phi, const void* d_ux, const void* d_uy,
                      const void* d_T, const void* d_p, int in_dtype, int mode)
{
    int rc = check_instance(c, instance);
    if (rc) return rc;
    if (!d_phi || !d_ux || !d_uy || !d_T) return fail(LBM_EINVAL, "NULL field");
    if (in_dtype != LBM_OUT_F64 && in_dtype != LBM_OUT_F32) return fail(LBM_EINVAL, "unknown input dtype");
    if (mode != LBM_REINIT_EQUILIBRIUM && mode != LBM_REINIT_SHIFT) return fail(LBM_EINVAL, "unknown reinit mode");
    const Layout& L = c->lay[instance];
    const lbm_params& p = c->params[instance];
    const long long n = (long long)L.nx * L.ny;
    const int lvl = (int)(c->step & 1);
    const size_t isz = inst_size(c->prec);
    const void* inst = static_cast<char*>(c->d_insts) + instance * isz;
    const int ft = lbm::grid_tile(c->tile);
    const lbm::Tile* tiles = c->d_tiles[ft] + L.tile_off[ft];
    // the other time level is free until the next step: it holds the staged
    // new fields (planes 0..4) and, when shifting, the current ones (5..9)
    double* staged = reinterpret_cast<double*>(c->ws + L.pop_off[lvl ^ 1]);
    HIP_TRY(lbm::launch_stage(d_phi, d_ux, d_uy, d_T, d_p, in_dtype == LBM_OUT_F32, n, staged, c->stream));
    if (mode == LBM_REINIT_SHIFT)
        HIP_TRY(lbm::launch_fields((int)c->prec, ft, c->d_insts, tiles, L.tile_cnt[ft], lvl, staged + 5 * n,
                                   staged + 6 * n, staged + 7 * n, staged + 8 * n, staged + 9 * n, 0, 0, c->stream));
    lbm::InitArgs ia{p.phi0_dev, p.T0_dev, 0.5 * (p.rho_l + p.rho_h), 0.5 * (p.rho_h - p.rho_l), d_p != nullptr,
                     mode == LBM_REINIT_SHIFT};
    HIP_TRY(lbm::launch_init((int)c->prec, inst, n, staged, ia, lvl, c->stream));
    HIP_TRY(lbm::launch_fields((int)c->prec, ft, c->d_insts, tiles, L.tile_cnt[ft], lvl, nullptr, nullptr,
                               nullptr, nullptr, nullptr, 0, 1, c->stream));
    return LBM_OK;
}

int lbm_fields(lbm_ctx* c, void* d_phi, void* d_ux, void* d_uy, void* d_T, void* d_p, int out_dtype)
{
    return lbm_fields_instance(c, 0, d_phi, d_ux, d_uy, d_T, d_p, out_dtype);
}

int lbm_diagnostics_instance(lbm_ctx* c, int instance, lbm_diag* out)
{
    int rc = check_instance(c, instance);
    if (rc) return rc;
    if (!out) return fail(LBM_EINVAL, "out is NULL");
    const Layout& L = c->lay[instance];
    const lbm_params& p = c->params[instance];
    lbm::DiagArgs a{};
    a.n_bubbles = (int)p.n_bubbles;
    for (int b = 0; b < 4; ++b) {
        a.bx[b] = c->bx[4 * instance + b];
        a.by[b] = c->by[4 * instance + b];
    }
    a.rcp_a = 0.5 * (p.rhocp_l + p.rhocp_h);
    a.rcp_b = 0.5 * (p.rhocp_h - p.rhocp_l);
    const int ft = lbm::grid_tile(c->tile);
    HIP_TRY(lbm::launch_diag((int)c->prec, ft, c->d_insts, c->d_tiles[ft] + L.tile_off[ft],
                             L.tile_cnt[ft], (int)(c->step & 1), a, c->d_partials, c->d_result, c->stream));
    double r[lbm::D_COUNT];
    HIP_TRY(hipMemcpyAsync(r, c->d_result, sizeof(r), hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    std::memset(out, 0, sizeof(*out));
    out->step = c->step;
    out->mass_phi = r[lbm::D_MASS];
    out->vol_light = r[lbm::D_VOL];
    out->heat = r[lbm::D_HEAT];
    out->sum_neg = r[lbm::D_SNEG];
    out->max_u = r[lbm::D_MAXU];
    out->n_nonfinite = (int64_t)r[lbm::D_NONFIN];
    out->n_neg = (int64_t)r[lbm::D_NNEG];
    if (out->sum_neg != 0.0) {
        out->u_r = r[lbm::D_SUY] / out->sum_neg;
        out->ux_r = r[lbm::D_SUX] / out->sum_neg;
        out->xc = r[lbm::D_SX] / out->sum_neg;
        out->yc = r[lbm::D_SY] / out->sum_neg;
    }
    for (int b = 0; b < (int)p.n_bubbles; ++b) {
        const double* q = r + lbm::D_BUB + 5 * b;
        out->bub_sum[b] = q[0];
        if (q[0] != 0.0) {
            out->bub_x[b] = q[1] / q[0];
            out->bub_y[b] = q[2] / q[0];
            out->bub_ux[b] = q[3] / q[0];
            out->bub_uy[b] = q[4] / q[0];
            c->bx[4 * instance + b] = out->bub_x[b];
            c->by[4 * instance + b] = out->bub_y[b];
        } else {
            out->bub_x[b] = c->bx[4 * instance + b];
            out->bub_y[b] = c->by[4 * instance + b];
        }
    }
    if (out->n_nonfinite > 0 || !(out->max_u <= 0.5))
        return fail(LBM_EUNSTABLE, "unstable: %lld non-finite nodes, max |u| = %g", (long long)out->n_nonfinite,
                    out->max_u);
    return LBM_OK;
}

int lbm_diagnostics(lbm_ctx* c, lbm_diag* out) { return lbm_diagnostics_instance(c, 0, out); }

int lbm_destroy(lbm_ctx* c)
{
    if (!c) return LBM_OK;
    hipError_t e = hipStreamSynchronize(c->stream);
    drop_graph(c);
    delete c;
    if (e != hipSuccess) return fail(LBM_EHIP, "hipStreamSynchronize: %s", hipGetErrorString(e));
    return LBM_OK;
}

const char* lbm_last_error(void) { return g_err.c_str(); }

// ---- state transfer ----

int lbm_get_state(lbm_ctx* c, int instance, double* f, double* g, double* h, double* jprev, int64_t* step)
{
    int rc = check_instance(c, instance);
    if (rc) return rc;
    const Layout& L = c->lay[instance];
    const lbm_params& p = c->params[instance];
    const size_t rsz = real_size(c->prec);
    const size_t nn = (size_t)L.nx * L.ny;
    const int lvl = (int)(c->step & 1);
    const size_t level_b = (size_t)lbm::kPlanes * L.plane * rsz;
    std::vector<char> lev(level_b), buf((size_t)L.plane * rsz);
    HIP_TRY(hipMemcpyAsync(lev.data(), c->ws + L.pop_off[lvl], level_b, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    // population q (q >= 0) from the level copy, or the plane at byte offset
    // off (q < 0)
    auto fetch = [&](int q, size_t off, double* dst, double shift_per_w, int k) -> int {
        if (q < 0) {
            HIP_TRY(hipMemcpyAsync(buf.data(), c->ws + off, buf.size(), hipMemcpyDeviceToHost, c->stream));
            HIP_TRY(hipStreamSynchronize(c->stream));
        }
        const char* src = q < 0 ? buf.data() : lev.data();
        const double sh = k >= 0 ? W9[k] * shift_per_w : 0.0;
        for (int j = 0; j < L.ny; ++j)
            for (int i = 0; i < L.nx; ++i) {
                const size_t n0 = (size_t)j * L.pitch + i;
                const size_t s = q < 0 ? n0 : (size_t)lbm::pop_index(q, (long long)n0);
                const double v = rsz == 8 ? reinterpret_cast<const double*>(src)[s]
                                          : (double)reinterpret_cast<const float*>(src)[s];
                dst[(size_t)j * L.nx + i] = v + sh;
            }
        return LBM_OK;
    };
    const size_t plane_b = (size_t)L.plane * rsz;
    for (int k = 0; k < 9; ++k) {
        if (f && (rc = fetch(lbm::kF + k, 0, f + k * nn, p.phi0_dev, k))) return rc;
        if (g && (rc = fetch(lbm::kG + k, 0, g + k * nn, 0.0, k))) return rc;
        if (h && (rc = fetch(lbm::kH + k, 0, h + k * nn, p.T0_dev, k))) return rc;
    }
    if (jprev)
        for (int q = 0; q < 2; ++q)
            if ((rc = fetch(-1, L.jprev_off + q * plane_b, jprev + q * nn, 0.0, -1))) return rc;
    if (step) *step = c->step;
    return LBM_OK;
}

int lbm_set_state(lbm_ctx* c, int instance, const double* f, const double* g, const double* h, const double* jprev,
                  int64_t step)
{
    int rc = check_instance(c, instance);
    if (rc) return rc;
    if (step < 0) return fail(LBM_EINVAL, "negative step");
    if (c->n > 1 && (step & 1) != (c->step & 1))
        return fail(LBM_EINVAL, "batched lattices share one time level: step parity must stay %lld",
                    (long long)(c->step & 1));
    const Layout& L = c->lay[instance];
    const lbm_params& p = c->params[instance];
    const size_t rsz = real_size(c->prec);
    const size_t nn = (size_t)L.nx * L.ny;
    // the current level is the one the new step count points at; copy the
    // other populations across if the parity changes
    const int old_lvl = (int)(c->step & 1), new_lvl = (int)(step & 1);
    const size_t level_b = (size_t)lbm::kPlanes * L.plane * rsz;
    if (old_lvl != new_lvl) {
        HIP_TRY(hipMemcpyAsync(c->ws + L.pop_off[new_lvl], c->ws + L.pop_off[old_lvl], level_b,
                               hipMemcpyDeviceToDevice, c->stream));
    }
    // the new level on the host (populations not given keep their values)
    std::vector<char> lev(level_b), buf((size_t)L.plane * rsz, 0);
    HIP_TRY(hipMemcpyAsync(lev.data(), c->ws + L.pop_off[new_lvl], level_b, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    // population q (q >= 0) into the level copy, or the plane at byte offset
    // off (q < 0, copied at once)
    auto put = [&](int q, size_t off, const double* srcp, double shift_per_w, int k) -> int {
        char* dst = q < 0 ? buf.data() : lev.data();
        const double sh = k >= 0 ? W9[k] * shift_per_w : 0.0;
        for (int j = 0; j < L.ny; ++j)
            for (int i = 0; i < L.nx; ++i) {
                const size_t n0 = (size_t)j * L.pitch + i;
                const size_t d = q < 0 ? n0 : (size_t)lbm::pop_index(q, (long long)n0);
                const double v = srcp[(size_t)j * L.nx + i] - sh;
                if (rsz == 8) reinterpret_cast<double*>(dst)[d] = v;
                else reinterpret_cast<float*>(dst)[d] = (float)v;
            }
        if (q < 0) {
            HIP_TRY(hipMemcpyAsync(c->ws + off, buf.data(), buf.size(), hipMemcpyHostToDevice, c->stream));
            HIP_TRY(hipStreamSynchronize(c->stream));
        }
        return LBM_OK;
    };
    const size_t plane_b = (size_t)L.plane * rsz;
    for (int k = 0; k < 9; ++k) {
        if (f && (rc = put(lbm::kF + k, 0, f + k * nn, p.phi0_dev, k))) return rc;
        if (g && (rc = put(lbm::kG + k, 0, g + k * nn, 0.0, k))) return rc;
        if (h && (rc = put(lbm::kH + k, 0, h + k * nn, p.T0_dev, k))) return rc;
    }
    HIP_TRY(hipMemcpyAsync(c->ws + L.pop_off[new_lvl], lev.data(), level_b, hipMemcpyHostToDevice, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    if (jprev)
        for (int q = 0; q < 2; ++q)
            if ((rc = put(-1, L.jprev_off + q * plane_b, jprev + q * nn, 0.0, -1))) return rc;
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->step = step;
    return LBM_OK;
}

namespace {
struct CkptHeader {
    char magic[8];
    uint32_t version, prec;
    int32_t n, pad;
    int64_t step;
    uint64_t hash;
    double bx[4], by[4];
};
size_t ckpt_payload(const lbm_ctx* c, int k)
{
    const size_t rsz = real_size(c->prec);
    return ((size_t)lbm::kPlanes + 2) * c->lay[k].plane * rsz;
}
}  // namespace

size_t lbm_checkpoint_bytes(const lbm_ctx* c)
{
    if (!c) return 0;
    size_t b = 0;
    for (int k = 0; k < c->n; ++k) b += sizeof(CkptHeader) + ckpt_payload(c, k);
    return b;
}

int lbm_checkpoint_save(lbm_ctx* c, void* host_buf, size_t bytes)
{
    if (!c || !host_buf) return fail(LBM_EINVAL, "NULL argument");
    if (bytes < lbm_checkpoint_bytes(c)) return fail(LBM_EINVAL, "checkpoint buffer too small");
    char* p = static_cast<char*>(host_buf);
    const uint64_t hsh = params_hash(c->params);
    const size_t rsz = real_size(c->prec);
    const int lvl = (int)(c->step & 1);
    for (int k = 0; k < c->n; ++k) {
        const Layout& L = c->lay[k];
        CkptHeader hd{};
        std::memcpy(hd.magic, "LBMCKPT3", 8);
        hd.version = LBM_ABI_VERSION;
        hd.prec = c->prec;
        hd.n = c->n;
        hd.step = c->step;
        hd.hash = hsh;
        for (int b = 0; b < 4; ++b) {
            hd.bx[b] = c->bx[4 * k + b];
            hd.by[b] = c->by[4 * k + b];
        }
        std::memcpy(p, &hd, sizeof(hd));
        p += sizeof(hd);
        const size_t level_b = (size_t)lbm::kPlanes * L.plane * rsz;
        HIP_TRY(hipMemcpyAsync(p, c->ws + L.pop_off[lvl], level_b, hipMemcpyDeviceToHost, c->stream));
        HIP_TRY(hipMemcpyAsync(p + level_b, c->ws + L.jprev_off, 2 * (size_t)L.plane * rsz, hipMemcpyDeviceToHost,
                               c->stream));
        p += ckpt_payload(c, k);
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    return LBM_OK;
}

int lbm_checkpoint_load(lbm_ctx* c, const void* host_buf, size_t bytes)
{
    if (!c || !host_buf) return fail(LBM_EINVAL, "NULL argument");
    if (bytes != lbm_checkpoint_bytes(c)) return fail(LBM_EINVAL, "checkpoint size %zu != %zu", bytes,
                                                      lbm_checkpoint_bytes(c));
    const char* p = static_cast<const char*>(host_buf);
    const uint64_t hsh = params_hash(c->params);
    const size_t rsz = real_size(c->prec);
    CkptHeader first{};
    std::memcpy(&first, p, sizeof(first));
    if (std::memcmp(first.magic, "LBMCKPT3", 8) || first.hash != hsh || first.prec != c->prec || first.n != c->n)
        return fail(LBM_EINVAL, "checkpoint of another format, or written by a context with different parameters");
    const int lvl = (int)(first.step & 1);
    for (int k = 0; k < c->n; ++k) {
        const Layout& L = c->lay[k];
        CkptHeader hd{};
        std::memcpy(&hd, p, sizeof(hd));
        p += sizeof(hd);
        for (int b = 0; b < 4; ++b) {
            c->bx[4 * k + b] = hd.bx[b];
            c->by[4 * k + b] = hd.by[b];
        }
        const size_t level_b = (size_t)lbm::kPlanes * L.plane * rsz;
        HIP_TRY(hipMemcpyAsync(c->ws + L.pop_off[lvl], p, level_b, hipMemcpyHostToDevice, c->stream));
        HIP_TRY(hipMemcpyAsync(c->ws + L.jprev_off, p + level_b, 2 * (size_t)L.plane * rsz, hipMemcpyHostToDevice,
                               c->stream));
        p += ckpt_payload(c, k);
    }
    HIP_TRY(hipStreamSynchronize(c->stream));
    c->step = first.step;
    return LBM_OK;
}

// ---- launch configuration ----

int lbm_tile_count(void) { return lbm::kTileCount; }

int lbm_tile_shape(int id, int* tx, int* ty)
{
    if (id < 0 || id >= lbm::kTileCount) return fail(LBM_EINVAL, "tile id %d out of range", id);
    // runs: tx = nodes per run, ty = 0
    const int rn = lbm::run_nodes(id);
    if (tx) *tx = rn ? rn : lbm::kTileTX[id];
    if (ty) *ty = rn ? 0 : lbm::kTileTY[id];
    return LBM_OK;
}

int lbm_set_tile(lbm_ctx* c, int id)
{
    if (!c) return fail(LBM_EINVAL, "context is NULL");
    if (id < 0 || id >= lbm::kTileCount) return fail(LBM_EINVAL, "tile id %d out of range", id);
    if (c->tile != id) {
        drop_graph(c);
        c->tile = id;
        if (c->n > 1) c->grid = -1;
    }
    return LBM_OK;
}

int lbm_get_tile(const lbm_ctx* c) { return c ? c->tile : -1; }

int lbm_set_graph_steps(lbm_ctx* c, int steps)
{
    if (!c) return fail(LBM_EINVAL, "context is NULL");
    if (steps < 0 || (steps & 1)) return fail(LBM_EINVAL, "graph steps must be even and >= 0");
    drop_graph(c);
    c->graph_steps = steps;
    return LBM_OK;
}

int lbm_set_grid(lbm_ctx* c, int workgroups)
{
    if (!c) return fail(LBM_EINVAL, "context is NULL");
    if (workgroups < 0) return fail(LBM_EINVAL, "negative grid");
    drop_graph(c);
    c->grid = workgroups > c->ntiles[c->tile] ? c->ntiles[c->tile] : workgroups;
    return LBM_OK;
}

int lbm_copy_probe(const void* d_src, void* d_dst, size_t bytes, void* hip_stream)
{
    if (!d_src || !d_dst || bytes == 0 || bytes % 16) return fail(LBM_EINVAL, "copy probe: bad arguments");
    if ((reinterpret_cast<uintptr_t>(d_src) | reinterpret_cast<uintptr_t>(d_dst)) % 16)
        return fail(LBM_EINVAL, "copy probe: buffers must be 16-byte aligned");
    HIP_TRY(lbm::launch_copy(d_src, d_dst, bytes, static_cast<hipStream_t>(hip_stream)));
    return LBM_OK;
}

int lbm_autotune(lbm_ctx* c, int steps_per_trial, int* best_tile, int* best_grid, float* best_ms)
{
    if (!c) return fail(LBM_EINVAL, "context is NULL");
    if (steps_per_trial < 1) return fail(LBM_EINVAL, "steps_per_trial must be >= 1");
    int dev = 0, cus = 0;
    HIP_TRY(hipGetDevice(&dev));
    HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    // Each trial replays a captured graph of G steps, as lbm_step does: the
    // graph of a configuration is captured and replayed once untimed, then
    // replayed once timed (plain launches would time the launch path of
    // small lattices rather than their kernels).
    const int saved_graph = c->graph_steps;
    const int G = steps_per_trial + (steps_per_trial & 1);
    drop_graph(c);
    c->graph_steps = G;
    float best = 1e30f;
    int bt = c->tile, bg = c->grid;
    // untimed steps first: the first candidate must not be timed on a cold
    // device (clocks and caches)
    int rc = lbm_step(c, G > 8 ? G : 8);
    if (rc == LBM_OK) {
        hipError_t e = hipStreamSynchronize(c->stream);
        if (e != hipSuccess) rc = fail(LBM_EHIP, "autotune warm-up: %s", hipGetErrorString(e));
    }
    for (int t = 0; t < lbm::kTileCount && rc == LBM_OK; ++t) {
        if (lbm::run_nodes(t) && !c->has_runs) continue;
        int grids[3] = {0, 0, 0}, ng = 1;
        if (c->n > 1) {
            int per_cu = 1;
            if (lbm::step_occupancy((int)c->prec, t, c->variant, &per_cu) != hipSuccess || per_cu < 1) per_cu = 1;
            const int resident = per_cu * (cus > 0 ? cus : 256);
            grids[0] = resident < c->ntiles[t] ? resident : c->ntiles[t];
            grids[1] = 2 * resident < c->ntiles[t] ? 2 * resident : c->ntiles[t];
            grids[2] = c->ntiles[t];
            ng = 3;
        }
        for (int q = 0; q < ng && rc == LBM_OK; ++q) {
            c->tile = t;
            c->grid = grids[q];
            drop_graph(c);
            // an even step count starts a graph; the untimed replay captures it
            if (c->step & 1) rc = lbm_step(c, 1);
            if (rc == LBM_OK) rc = lbm_step(c, G);
            if (rc) break;
            hipError_t e = hipEventRecord(e0, c->stream);
            if (e == hipSuccess) rc = lbm_step(c, G);
            if (rc) break;
            if (e == hipSuccess) e = hipEventRecord(e1, c->stream);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0.f;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e != hipSuccess) {
                rc = fail(LBM_EHIP, "autotune timing: %s", hipGetErrorString(e));
                break;
            }
            ms /= (float)G;
            if (ms < best) {
                best = ms;
                bt = t;
                bg = grids[q];
            }
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    drop_graph(c);
    c->tile = bt;
    c->grid = bg;
    c->graph_steps = saved_graph;
    if (rc) return rc;
    if (best_tile) *best_tile = bt;
    if (best_grid) *best_grid = bg;
    if (best_ms) *best_ms = best;
    return LBM_OK;
}

int lbm_get_grid(const lbm_ctx* c) { return c ? c->grid : -1; }

size_t lbm_bytes_per_update(int precision)
{
    const size_t rsz = precision == LBM_FP64 ? 8 : 4;
    return (2 * lbm::kPlanes + 4) * rsz;
}

}  // extern "C"
