/* Memory- and UB-checked run of the C oracle (test infrastructure): built
 * together with oracle/oracle.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer by tests/test_oracle_sanitize.py, it drives
 * every exported routine on small ragged grids with solid cells, walls, a
 * pressure axis and a body force, for every velocity set and collision the
 * oracle accepts.  Exit status 0 and "ok" on stdout when nothing fired. */
#include "../oracle/oracle.c"

#include <stdio.h>

static unsigned long long g_state = 88172645463325252ull;
static double urand(void) /* xorshift64, uniform in [0, 1) */
{
    g_state ^= g_state << 13;
    g_state ^= g_state >> 7;
    g_state ^= g_state << 17;
    return (double)(g_state >> 11) / 9007199254740992.0;
}

static int run_case(int q, int coll, int closure, const double *mlp)
{
    const int nx = 7, ny = 5, nz = 4, N = nx * ny * nz;
    double *rho = malloc(sizeof(double) * N), *u = malloc(sizeof(double) * 3 * N);
    double *d = malloc(sizeof(double) * q * N), *post = malloc(sizeof(double) * q * N);
    double *uv = malloc(sizeof(double) * 3 * N), *r2 = malloc(sizeof(double) * N);
    double *u2 = malloc(sizeof(double) * 3 * N), tot[8], fo[8];
    uint8_t *solid = malloc(N);
    for (int k = 0; k < N; ++k) {
        rho[k] = 1.0 + 0.01 * (urand() - 0.5);
        for (int a = 0; a < 3; ++a) u[a * N + k] = (q == 9 && a == 2) ? 0.0 : 0.02 * (urand() - 0.5);
        const int x = k % nx;
        solid[k] = (x > 0 && x < nx - 1 && urand() < 0.15) ? 1 : 0;
    }
    orc_params p;
    memset(&p, 0, sizeof p);
    p.q = q;
    p.collision = coll;
    p.tau = 0.7;
    p.magic = 3.0 / 16.0;
    p.omega_bulk = 1.2;
    p.omega_higher = 1.1;
    p.force[0] = 1e-5;
    p.force[1] = q == 9 ? 0.0 : -1e-6;
    p.closure = closure;
    p.cs_smag = 0.1;
    p.mlp = mlp;
    p.periodic[1] = 0;
    p.periodic[2] = 1;
    p.pressure_axis = 0;
    p.rho_in = 1.002;
    p.rho_out = 0.998;
    int rc = orc_init(q, nx, ny, nz, rho, u, solid, d);
    rc = rc ? rc : orc_run(&p, nx, ny, nz, solid, d, 3, 1);
    rc = rc ? rc : orc_collide(&p, nx, ny, nz, solid, d, post, uv, 1);
    rc = rc ? rc : orc_stream(&p, nx, ny, nz, solid, post, uv, d);
    rc = rc ? rc : orc_momentum_exchange(&p, nx, ny, nz, solid, post, fo);
    rc = rc ? rc : orc_moments(q, p.force, nx, ny, nz, solid, d, r2, u2, tot);
    double dc[OQ], dout[OQ], rut[5];
    for (int i = 0; i < q; ++i) dc[i] = d[i * N + N / 2];
    rc = rc ? rc : orc_collide_cell(&p, dc, dout, rut);
    free(rho), free(u), free(d), free(post), free(uv), free(r2), free(u2), free(solid);
    if (rc) fprintf(stderr, "case q%d coll%d closure%d: rc %d\n", q, coll, closure, rc);
    return rc;
}

int main(void)
{
    const int sets[4] = {9, 15, 19, 27};
    int fails = 0;
    double *P = malloc(sizeof(double) * ORC_MLP_NPARAM), *g = malloc(sizeof(double) * ORC_MLP_NPARAM);
    for (int k = 0; k < ORC_MLP_NPARAM; ++k) P[k] = 0.1 * (urand() - 0.5);
    for (int k = 7; k < 14; ++k) P[k] = 100.0; /* inv_std of the features */
    for (int s = 0; s < 4; ++s) {
        const int q = sets[s];
        int c[3 * OQ], opp[OQ];
        double w[OQ];
        if (orc_stencil(q, c, w, opp)) ++fails;
        for (int coll = 0; coll <= 4; ++coll) {
            const int valid = coll <= 1 || (coll == 2 && q >= 19) || (coll >= 3 && q == 27);
            if (!valid) continue;
            fails += run_case(q, coll, 0, NULL) != 0;
            fails += run_case(q, coll, 1, NULL) != 0;
        }
        if (q >= 19) {
            double M[OQ * OQ], Mi[OQ * OQ];
            int kind[OQ];
            if (orc_mlp_nparam() != ORC_MLP_NPARAM || orc_mrt_matrix(q, M, Mi, kind)) ++fails;
        }
    }
    fails += run_case(19, 1, 2, P) != 0; /* learned closure */
    double raw[7 * 16], o[16], t[16], loss = 0.0;
    int32_t flag[16];
    for (int k = 0; k < 7 * 16; ++k) raw[k] = 1e-3 * (urand() - 0.5);
    for (int k = 0; k < 16; ++k) t[k] = urand();
    fails += orc_mlp_forward(P, 16, raw, o, flag) != 0;
    fails += orc_mlp_backward(P, 16, raw, t, 1.0, g, &loss) != 0;
    free(P), free(g);
    if (fails) return 1;
    printf("ok\n");
    return 0;
}
