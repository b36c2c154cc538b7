/* Runs the FP64 oracle on tiny lattices under the address and undefined-
 * behaviour sanitizers (built by tests/test_oracle_sanitize.py with gcc).
 * Every boundary combination, both collision models, both force forms, both
 * normal modes and tracked regions are stepped; each state must stay finite
 * and every slot of the new level must be written exactly once. */
#include "../../oracle/lbm_oracle.c"

#include <stdio.h>

static int run_case(int nx, int ny, const int bc[4], int grad_mode, int collision, int force_form, int steps)
{
    orc_params P;
    memset(&P, 0, sizeof(P));
    P.nx = nx;
    P.ny = ny;
    for (int s = 0; s < 4; ++s) P.bc[s] = bc[s];
    P.grad_mode = grad_mode;
    P.collision = collision;
    P.force_form = force_form;
    P.trt_magic = 3.0 / 16.0;
    P.n_bubbles = 2;
    P.bubble_x[0] = 0.3 * nx; P.bubble_y[0] = 0.5 * ny;
    P.bubble_x[1] = 0.7 * nx; P.bubble_y[1] = 0.5 * ny;
    P.rho_l = 0.4; P.rho_h = 1.0; P.mu_l = 0.05; P.mu_h = 0.1;
    P.lam_l = 0.2; P.lam_h = 0.1; P.rcp_l = 1.0; P.rcp_h = 2.0;
    P.sigma_ref = 1e-2; P.sigma_T = -1e-3; P.sigma_TT = 2e-3; P.T_ref = 0.5;
    P.W = 2.0; P.M = 0.1; P.Gx = 1e-6; P.Gy = -2e-6;
    for (int s = 0; s < 4; ++s) { P.tw_mean[s] = 0.25 * s; P.tw_amp[s] = 0.1; P.tw_k[s] = 0.3; P.tw_slope[s] = 0.01; }
    P.u_in = 1e-3; P.phi_in = 1.0; P.T_in = 0.2;
    const size_t n = (size_t)nx * ny;
    double* phi = malloc(n * sizeof(double));
    double* ux = malloc(n * sizeof(double));
    double* uy = malloc(n * sizeof(double));
    double* T = malloc(n * sizeof(double));
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const size_t x = (size_t)j * nx + i;
            const double r = hypot(i - 0.5 * nx, j - 0.5 * ny) - 0.3 * (nx < ny ? nx : ny);
            phi[x] = tanh(r / (sqrt(2.0) * P.W));
            ux[x] = 1e-3 * sin(0.7 * i + 0.3 * j);
            uy[x] = -1e-3 * cos(0.2 * i - 0.5 * j);
            T[x] = 0.5 + 0.1 * sin(0.4 * i) * cos(0.6 * j);
        }
    orc_state* S = orc_create(&P, phi, ux, uy, T);
    int bad = 0;
    if (!S) { fprintf(stderr, "create failed\n"); bad = 1; goto out; }
    orc_step(S, steps);
    int* cnt = malloc(9 * n * sizeof(int));
    if (orc_step_count_writes(S, cnt) != 0) bad = 1;
    for (size_t q = 0; q < 9 * n && !bad; ++q)
        if (cnt[q] != 1) { fprintf(stderr, "slot %zu written %d times\n", q, cnt[q]); bad = 1; }
    free(cnt);
    double* buf = malloc(13 * n * sizeof(double));
    orc_macros_all(S, buf);
    for (size_t q = 0; q < 13 * n && !bad; ++q)
        if (!isfinite(buf[q])) { fprintf(stderr, "non-finite macro %zu\n", q); bad = 1; }
    free(buf);
    orc_diag D;
    orc_diagnostics(S, &D);
    if (D.n_nonfinite) bad = 1;
    orc_fields(S, phi, ux, uy, T, T);
    orc_destroy(S);
out:
    free(phi); free(ux); free(uy); free(T);
    return bad;
}

int main(void)
{
    static const int bcs[][4] = {
        {0, 0, 0, 0}, {0, 0, 1, 1}, {0, 0, 2, 1}, {1, 1, 2, 2}, {1, 1, 3, 4}, {2, 2, 3, 4}, {3, 4, 1, 1}, {1, 2, 1, 2}};
    static const int sizes[][2] = {{5, 4}, {9, 7}, {16, 11}};
    int fails = 0, cases = 0;
    for (size_t b = 0; b < sizeof(bcs) / sizeof(bcs[0]); ++b)
        for (size_t z = 0; z < sizeof(sizes) / sizeof(sizes[0]); ++z)
            for (int v = 0; v < 4; ++v) {
                const int grad_mode = v & 1, collision = (v >> 1) & 1, force_form = (int)((b + z + v) & 1);
                fails += run_case(sizes[z][0], sizes[z][1], bcs[b], grad_mode, collision, force_form, 6);
                ++cases;
            }
    printf("cases %d failures %d\n", cases, fails);
    return fails ? 1 : 0;
}
