/*
 * oracle.c -- plain FP64 CPU reference of the lattice Boltzmann update.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness oracle for the
 * HIP library.  Only the test suite, the smoke check and the CPU-baseline leg
 * of the benchmark load it.  It shares no source, header, table or helper
 * with the GPU path, and the GPU path never loads it.
 *
 * What it computes (paper: Bauer et al., "waLBerla: A block-structured
 * high-performance framework for multiphysics simulations", Sec. 5.1.1):
 *   - moments rho = sum_i f_i, rho*u = sum_i c_i f_i               (Eq. 1)
 *   - update f_i(x + c_i, t + 1) = f_i(x, t) + Omega_i(f(x, t)):
 *     collision, then streaming to the neighbour                   (Eq. 2)
 *   - MRT collision Omega = -M^{-1} S (M f - m_eq)                   (Eq. 3)
 *     with SRT and TRT as special choices of S (Sec. 5.1.1), and the KBC
 *     entropic stabilisation as a per-cell choice of the higher rates
 *     (Sec. 5.1.1, Boesch et al. 2015), and the cumulant collision
 *     (Sec. 5.1.1, Geier et al. 2015)
 *   - locally varying relaxation time from a closure (Sec. 5.1.1,
 *     turbulence models after Yu et al. 2005)
 *   - no-slip / pressure boundaries and body-force driving (Sec. 5.1.1,
 *     Ginzburg et al. 2008; Guo et al. 2002)
 *   - the force on obstacles by momentum exchange (Sec. "Geometrically fully
 *     resolved simulations"; Ladd 1994, Aidun et al. 1998)
 *
 * Deliberately NOT the GPU's scheme: one global lattice, no blocks, no ghost
 * layers, two arrays, "pull" streaming.  State is the deviation
 * d_i = f_i - w_i (rho - 1 = sum d_i, j = sum c_i d_i exactly, because
 * sum w_i = 1 and sum w_i c_i = 0).  Solid cells carry no state (d = 0).
 *
 * Readings where the paper gives a name but not a formula:
 *   velocity sets, weights, c_s^2 = 1/3: textbook D2Q9/D3Q15/D3Q19/D3Q27
 *        (Krueger 2017); MRT, KBC and cumulant only on D3Q19/D3Q27;
 *   equilibrium: second-order polynomial f_eq (same for every set);
 *   force: Guo 2002 term, u = (sum c f + F/2)/rho;
 *   TRT: Lambda = (tau+ - 1/2)(tau- - 1/2) (Ginzburg 2008);
 *   MRT: raw-moment monomial basis c_x^a c_y^b c_z^c, second-order
 *        diagonal rows recombined into x2-y2, x2-z2, x2+y2+z2;
 *   walls: half-way bounce-back; pressure: anti-bounce-back;
 *   Smagorinsky: tau from |Pi_neq| in closed form (Yu 2005);
 *   MLP closure: 7 -> 32 -> 32 -> 1, erf-GELU, softplus output, bf16 GEMM
 *        operands, fp32 parameters (evaluated here in FP64).
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fPIC -shared
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OQ 27 /* largest velocity set */

/* ------------------------------------------------------------------------ */
/* Parameters                                                               */
/* ------------------------------------------------------------------------ */
typedef struct {
    int q;                /* 9, 15, 19 or 27 */
    int collision;        /* 0 = SRT, 1 = TRT, 2 = MRT, 3 = KBC (MRT basis, entropic higher rates),
                             4 = cumulant (D3Q27) */
    double tau;           /* shear relaxation time tau_0 */
    double magic;         /* TRT magic parameter Lambda */
    double omega_bulk;    /* MRT rate of x2+y2+z2 */
    double omega_higher;  /* MRT rate of moments of order >= 3 */
    double force[3];      /* body force density F */
    int closure;          /* 0 = none, 1 = Smagorinsky, 2 = MLP */
    double cs_smag;       /* Smagorinsky constant C_s */
    const double *mlp;    /* packed MLP parameters (ORC_MLP_NPARAM), or NULL */
    int periodic[3];      /* per axis: 1 = periodic, 0 = walls (or pressure) */
    int pressure_axis;    /* -1 = none; otherwise that axis has density BCs */
    double rho_in;        /* density imposed at the low end of pressure_axis */
    double rho_out;       /* density imposed at the high end */
} orc_params;

/* ------------------------------------------------------------------------ */
/* Velocity sets (textbook, Krueger 2017; the paper names D2Q9, D3Q15,      */
/* D3Q19 and D3Q27 in Sec. 5.1.1)                                            */
/* ------------------------------------------------------------------------ */
/* Order: rest; the six axis directions as +/- pairs; the twelve edge
 * directions as +/- pairs; the eight corners as +/- pairs.  Each odd index
 * is followed by its opposite. */
static const int C27[OQ][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
    {1, 1, 1}, {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
    {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1},
};

/* D3Q15: rest, the six axis directions, the eight corners (same pairs and
 * order as in C27).  D2Q9: rest, (+-1,0), (0,+-1), then (1,1), (-1,-1),
 * (1,-1), (-1,1); the third component is 0, so a 3D grid holds independent
 * 2D planes. */
static const int C15[15][3] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 1}, {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
    {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1},
};
static const int C9[9][3] = {
    {0, 0, 0}, {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
};

typedef struct {
    int q;
    int c[OQ][3];
    double w[OQ];
    int opp[OQ];
} lattice;

static int make_lattice(int q, lattice *L)
{
    if (q != 9 && q != 15 && q != 19 && q != 27) return -1;
    L->q = q;
    for (int i = 0; i < q; ++i) {
        const int *ci = q == 9 ? C9[i] : (q == 15 ? C15[i] : C27[i]);
        int n2 = 0;
        for (int a = 0; a < 3; ++a) {
            L->c[i][a] = ci[a];
            n2 += ci[a] * ci[a];
        }
        if (q == 9) {
            /* D2Q9: 4/9, 1/9, 1/36 for |c|^2 = 0, 1, 2 */
            L->w[i] = n2 == 0 ? 4.0 / 9.0 : (n2 == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
        } else if (q == 15) {
            /* D3Q15: 2/9, 1/9, 1/72 for |c|^2 = 0, 1, 3 */
            L->w[i] = n2 == 0 ? 2.0 / 9.0 : (n2 == 1 ? 1.0 / 9.0 : 1.0 / 72.0);
        } else if (q == 27) {
            /* D3Q27 weights: product of the D1Q3 weights 2/3 (rest) and 1/6,
             * i.e. 2^(3 - 2 |c|^2) / 27 = 8/27, 2/27, 1/54, 1/216. */
            L->w[i] = ldexp(1.0, 3 - 2 * n2) / 27.0;
        } else {
            L->w[i] = (n2 == 0) ? 1.0 / 3.0 : (n2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
        }
    }
    /* opposite: the direction with c -> -c */
    for (int i = 0; i < q; ++i) {
        L->opp[i] = -1;
        for (int k = 0; k < q; ++k)
            if (L->c[k][0] == -L->c[i][0] && L->c[k][1] == -L->c[i][1] && L->c[k][2] == -L->c[i][2])
                L->opp[i] = k;
    }
    return 0;
}

int orc_stencil(int q, int *c_out, double *w_out, int *opp_out)
{
    lattice L;
    if (make_lattice(q, &L)) return -1;
    for (int i = 0; i < q; ++i) {
        for (int a = 0; a < 3; ++a) c_out[3 * i + a] = L.c[i][a];
        w_out[i] = L.w[i];
        opp_out[i] = L.opp[i];
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* MRT moment matrix (Eq. 3): rows are raw moments sum_i c_x^a c_y^b c_z^c f_i */
/* ------------------------------------------------------------------------ */
typedef struct {
    int q;
    double M[OQ][OQ];
    double Minv[OQ][OQ];
    int kind[OQ]; /* 0 conserved, 1 shear, 2 bulk, 3 higher */
} mrt_basis;

static double ipow(int c, int e)
{
    double r = 1.0;
    for (int k = 0; k < e; ++k) r *= c;
    return r;
}

/* Gauss-Jordan inversion with partial pivoting, FP64. */
static int invert(int n, double A[OQ][OQ], double Ainv[OQ][OQ])
{
    double W[OQ][2 * OQ];
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < 2 * n; ++c)
            W[r][c] = (c < n) ? A[r][c] : (c - n == r ? 1.0 : 0.0);
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(W[r][col]) > fabs(W[piv][col])) piv = r;
        if (fabs(W[piv][col]) < 1e-12) return -1;
        if (piv != col)
            for (int c = 0; c < 2 * n; ++c) {
                double t = W[piv][c];
                W[piv][c] = W[col][c];
                W[col][c] = t;
            }
        double p = W[col][col];
        for (int c = 0; c < 2 * n; ++c) W[col][c] /= p;
        for (int r = 0; r < n; ++r) {
            if (r == col) continue;
            double f = W[r][col];
            if (f == 0.0) continue;
            for (int c = 0; c < 2 * n; ++c) W[r][c] -= f * W[col][c];
        }
    }
    for (int r = 0; r < n; ++r)
        for (int c = 0; c < n; ++c) Ainv[r][c] = W[r][c + n];
    return 0;
}

static int make_mrt(const lattice *L, mrt_basis *B)
{
    int q = L->q, row = 0;
    int ex[OQ][3];
    for (int c = 0; c < 3; ++c)
        for (int b = 0; b < 3; ++b)
            for (int a = 0; a < 3; ++a) {
                if (q == 19 && a > 0 && b > 0 && c > 0) continue; /* no xyz factor */
                ex[row][0] = a;
                ex[row][1] = b;
                ex[row][2] = c;
                ++row;
            }
    if (row != q) return -1;
    B->q = q;
    int rxx = -1, ryy = -1, rzz = -1;
    for (int r = 0; r < q; ++r) {
        int a = ex[r][0], b = ex[r][1], c = ex[r][2];
        for (int i = 0; i < q; ++i)
            B->M[r][i] = ipow(L->c[i][0], a) * ipow(L->c[i][1], b) * ipow(L->c[i][2], c);
        int order = a + b + c;
        if (order <= 1) B->kind[r] = 0;
        else if (order == 2 && (a == 2 || b == 2 || c == 2)) B->kind[r] = -1; /* diagonal, fixed below */
        else if (order == 2) B->kind[r] = 1;
        else B->kind[r] = 3;
        if (a == 2 && b == 0 && c == 0) rxx = r;
        if (a == 0 && b == 2 && c == 0) ryy = r;
        if (a == 0 && b == 0 && c == 2) rzz = r;
    }
    /* recombine the three diagonal second-order rows */
    double xx[OQ], yy[OQ], zz[OQ];
    for (int i = 0; i < q; ++i) {
        xx[i] = B->M[rxx][i];
        yy[i] = B->M[ryy][i];
        zz[i] = B->M[rzz][i];
    }
    for (int i = 0; i < q; ++i) {
        B->M[rxx][i] = xx[i] - yy[i];
        B->M[ryy][i] = xx[i] - zz[i];
        B->M[rzz][i] = xx[i] + yy[i] + zz[i];
    }
    B->kind[rxx] = 1;
    B->kind[ryy] = 1;
    B->kind[rzz] = 2;
    return invert(q, B->M, B->Minv);
}

int orc_mrt_matrix(int q, double *M_out, double *Minv_out, int *kind_out)
{
    lattice L;
    mrt_basis B;
    if (make_lattice(q, &L) || make_mrt(&L, &B)) return -1;
    for (int r = 0; r < q; ++r) {
        kind_out[r] = B.kind[r];
        for (int c = 0; c < q; ++c) {
            M_out[r * q + c] = B.M[r][c];
            Minv_out[r * q + c] = B.Minv[r][c];
        }
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Learned closure: per-cell MLP (evaluated in FP64, bf16 operand rounding)  */
/* ------------------------------------------------------------------------ */
#define ORC_MLP_IN 7
#define ORC_MLP_H 32
#define ORC_MLP_OFF_MEAN 0
#define ORC_MLP_OFF_ISTD 7
#define ORC_MLP_OFF_W1 14
#define ORC_MLP_OFF_B1 (ORC_MLP_OFF_W1 + ORC_MLP_H * ORC_MLP_IN)
#define ORC_MLP_OFF_W2 (ORC_MLP_OFF_B1 + ORC_MLP_H)
#define ORC_MLP_OFF_B2 (ORC_MLP_OFF_W2 + ORC_MLP_H * ORC_MLP_H)
#define ORC_MLP_OFF_W3 (ORC_MLP_OFF_B2 + ORC_MLP_H)
#define ORC_MLP_OFF_B3 (ORC_MLP_OFF_W3 + ORC_MLP_H)
#define ORC_MLP_NPARAM (ORC_MLP_OFF_B3 + 1)

/* Round to single precision, then to bfloat16 with round-to-nearest-even on
 * the 16 dropped mantissa bits.  This is where the GPU feeds its GEMMs. */
static int g_bf16 = 1; /* 0 only for finite-difference checks of the backward pass */

void orc_mlp_set_rounding(int on) { g_bf16 = on; }

static double to_bf16(double v)
{
    if (!g_bf16) return v;
    float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) { /* inf / nan unchanged (quiet nan) */
        if (u & 0x007fffffu) u |= 0x00400000u;
        u &= 0xffff0000u;
    } else {
        uint32_t lsb = (u >> 16) & 1u;
        u = (u + 0x7fffu + lsb) & 0xffff0000u;
    }
    memcpy(&f, &u, 4);
    return (double)f;
}

double orc_bf16_round(double v)
{
    int keep = g_bf16;
    g_bf16 = 1;
    double r = to_bf16(v);
    g_bf16 = keep;
    return r;
}


static double gelu(double z) { return 0.5 * z * (1.0 + erf(z / sqrt(2.0))); }
static double gelu_grad(double z)
{
    return 0.5 * (1.0 + erf(z / sqrt(2.0))) + z * exp(-0.5 * z * z) / sqrt(2.0 * M_PI);
}
static double softplus(double o) { return o > 30.0 ? o : log1p(exp(o)); }
static double sigmoid(double o) { return 1.0 / (1.0 + exp(-o)); }

double orc_gelu(double z) { return gelu(z); }
double orc_softplus(double o) { return softplus(o); }

/* Standardised features x_k = (raw_k - mean_k) * inv_std_k.  Returns 1 when a
 * feature is out of the trusted range |x_k| > 8 (closure falls back). */
static int mlp_features(const double *P, const double *raw, double *x)
{
    int bad = 0;
    for (int k = 0; k < ORC_MLP_IN; ++k) {
        x[k] = (raw[k] - P[ORC_MLP_OFF_MEAN + k]) * P[ORC_MLP_OFF_ISTD + k];
        if (!(fabs(x[k]) <= 8.0)) bad = 1;
    }
    return bad;
}

/* Forward pass; z1/h1/z2/h2 may be NULL.  Returns the scalar output o. */
static double mlp_forward(const double *P, const double *x, double *z1, double *h1,
                          double *z2, double *h2)
{
    double xb[ORC_MLP_IN], a1[ORC_MLP_H], a2[ORC_MLP_H], g1[ORC_MLP_H], g2[ORC_MLP_H];
    for (int k = 0; k < ORC_MLP_IN; ++k) xb[k] = to_bf16(x[k]);
    for (int j = 0; j < ORC_MLP_H; ++j) {
        double s = 0.0;
        for (int k = 0; k < ORC_MLP_IN; ++k) s += to_bf16(P[ORC_MLP_OFF_W1 + j * ORC_MLP_IN + k]) * xb[k];
        a1[j] = s + P[ORC_MLP_OFF_B1 + j];
        g1[j] = gelu(a1[j]);
    }
    for (int j = 0; j < ORC_MLP_H; ++j) {
        double s = 0.0;
        for (int k = 0; k < ORC_MLP_H; ++k) s += to_bf16(P[ORC_MLP_OFF_W2 + j * ORC_MLP_H + k]) * to_bf16(g1[k]);
        a2[j] = s + P[ORC_MLP_OFF_B2 + j];
        g2[j] = gelu(a2[j]);
    }
    double o = 0.0;
    for (int k = 0; k < ORC_MLP_H; ++k) o += to_bf16(P[ORC_MLP_OFF_W3 + k]) * to_bf16(g2[k]);
    o += P[ORC_MLP_OFF_B3];
    if (z1) memcpy(z1, a1, sizeof a1);
    if (h1) memcpy(h1, g1, sizeof g1);
    if (z2) memcpy(z2, a2, sizeof a2);
    if (h2) memcpy(h2, g2, sizeof g2);
    return o;
}

/* Batched forward: raw[n][7] -> o[n]; flag[n] = 1 where the fallback applies. */
int orc_mlp_forward(const double *P, int64_t n, const double *raw, double *o, int32_t *flag)
{
    for (int64_t s = 0; s < n; ++s) {
        double x[ORC_MLP_IN];
        int bad = mlp_features(P, raw + ORC_MLP_IN * s, x);
        o[s] = mlp_forward(P, x, NULL, NULL, NULL, NULL);
        if (flag) flag[s] = bad || !isfinite(o[s]);
    }
    return 0;
}

/* Forward pass with the rounded operands of one rounding point replaced:
 * layer 0 = input x_k, 1 = first hidden h1_k, 2 = second hidden h2_k (the
 * values fed to the GEMMs); layer -1 replaces nothing. */
static double mlp_forward_replace(const double *P, const double *x, int layer, int idx, double val)
{
    double xb[ORC_MLP_IN], g1[ORC_MLP_H], g2[ORC_MLP_H];
    for (int k = 0; k < ORC_MLP_IN; ++k) xb[k] = to_bf16(x[k]);
    if (layer == 0) xb[idx] = val;
    for (int j = 0; j < ORC_MLP_H; ++j) {
        double s = 0.0;
        for (int k = 0; k < ORC_MLP_IN; ++k) s += to_bf16(P[ORC_MLP_OFF_W1 + j * ORC_MLP_IN + k]) * xb[k];
        g1[j] = to_bf16(gelu(s + P[ORC_MLP_OFF_B1 + j]));
    }
    if (layer == 1) g1[idx] = val;
    for (int j = 0; j < ORC_MLP_H; ++j) {
        double s = 0.0;
        for (int k = 0; k < ORC_MLP_H; ++k) s += to_bf16(P[ORC_MLP_OFF_W2 + j * ORC_MLP_H + k]) * g1[k];
        g2[j] = to_bf16(gelu(s + P[ORC_MLP_OFF_B2 + j]));
    }
    if (layer == 2) g2[idx] = val;
    double o = 0.0;
    for (int k = 0; k < ORC_MLP_H; ++k) o += to_bf16(P[ORC_MLP_OFF_W3 + k]) * g2[k];
    return o + P[ORC_MLP_OFF_B3];
}

/* Distance of v from the nearest bf16 rounding boundary (a midpoint between
 * two adjacent bf16 values), and the bf16 value on the other side of it. */
static double bf16_boundary(double v, double *other)
{
    const double a = fabs(v);
    float fa = (float)a;
    uint32_t u;
    memcpy(&u, &fa, 4);
    const uint32_t lo = u & 0xffff0000u;
    double best = INFINITY, mid_best = 0.0;
    for (int k = 0; k < 2; ++k) {
        if (k == 1 && lo < 0x10000u) break;
        const uint32_t mb = (k == 0 ? lo : lo - 0x10000u) | 0x8000u;
        float fm;
        memcpy(&fm, &mb, 4);
        const double dist = fabs(a - (double)fm);
        if (dist < best) {
            best = dist;
            mid_best = (double)fm;
        }
    }
    /* reflect the rounded value across the midpoint */
    const double r = fabs(to_bf16(a));
    const double o = 2.0 * mid_best - r;
    *other = v < 0 ? -o : o;
    return best;
}

/* Rounding decisions of the network evaluated in single precision (the
 * GPU's matrix-core forward: standardisation in FP32, exact bf16 products
 * summed in FP32 in any order, GELU(z) with relative error at most
 * rel0 + rel2 z^2).  Such an
 * evaluation takes every bf16 rounding decision of this oracle the same way
 * unless the operand lies within the evaluation's error bound of a rounding
 * boundary.  Error bounds per operand (u = 2^-24; n-term sums bounded by
 * gamma_n = n u / (1 - n u) times the sum of magnitudes):
 *   x_k:  2u |x_k| (a subtraction and a product);
 *   h1_j: |GELU'(z)| gamma_8 (sum |W1 x| + |b1|) + (rel0 + rel2 z^2 + 2u) |h1|
 *         + 2^-126 (z the pre-activation);
 *   h2_j: the same with gamma_33 (sum |W2 h1| + |b2|);
 * each computed from this oracle's own (rounded) operands.  For every sample:
 * count[s] = number of undecided operands, flip[s] = sum over them of |o'-o|
 * with o' the output when that operand alone takes its other bf16 neighbour
 * (the layers after it recomputed). */
int orc_mlp_undecided(const double *P, int64_t n, const double *raw, double rel0, double rel2, int32_t *count,
                      double *flip)
{
    const double u = ldexp(1.0, -24);
    const double g8 = 8 * u / (1 - 8 * u), g33 = 33 * u / (1 - 33 * u);
    for (int64_t s = 0; s < n; ++s) {
        double x[ORC_MLP_IN], xb[ORC_MLP_IN], g1b[ORC_MLP_H];
        mlp_features(P, raw + ORC_MLP_IN * s, x);
        const double o = mlp_forward_replace(P, x, -1, 0, 0.0);
        int cnt = 0;
        double eff = 0.0, other;
        for (int k = 0; k < ORC_MLP_IN; ++k) {
            xb[k] = to_bf16(x[k]);
            if (bf16_boundary(x[k], &other) <= 2 * u * fabs(x[k])) {
                ++cnt;
                eff += fabs(mlp_forward_replace(P, x, 0, k, other) - o);
            }
        }
        for (int j = 0; j < ORC_MLP_H; ++j) {
            double sum = 0.0, mag = fabs(P[ORC_MLP_OFF_B1 + j]);
            for (int k = 0; k < ORC_MLP_IN; ++k) {
                const double t = to_bf16(P[ORC_MLP_OFF_W1 + j * ORC_MLP_IN + k]) * xb[k];
                sum += t;
                mag += fabs(t);
            }
            const double z = sum + P[ORC_MLP_OFF_B1 + j], h = gelu(z);
            g1b[j] = to_bf16(h);
            const double e = fabs(gelu_grad(z)) * g8 * mag + (rel0 + rel2 * z * z + 2 * u) * fabs(h) + ldexp(1.0, -126);
            if (bf16_boundary(h, &other) <= e) {
                ++cnt;
                eff += fabs(mlp_forward_replace(P, x, 1, j, other) - o);
            }
        }
        for (int j = 0; j < ORC_MLP_H; ++j) {
            double sum = 0.0, mag = fabs(P[ORC_MLP_OFF_B2 + j]);
            for (int k = 0; k < ORC_MLP_H; ++k) {
                const double t = to_bf16(P[ORC_MLP_OFF_W2 + j * ORC_MLP_H + k]) * g1b[k];
                sum += t;
                mag += fabs(t);
            }
            const double z = sum + P[ORC_MLP_OFF_B2 + j], h = gelu(z);
            const double e = fabs(gelu_grad(z)) * g33 * mag + (rel0 + rel2 * z * z + 2 * u) * fabs(h) + ldexp(1.0, -126);
            if (bf16_boundary(h, &other) <= e) {
                ++cnt;
                eff += fabs(mlp_forward_replace(P, x, 2, j, other) - o);
            }
        }
        count[s] = cnt;
        flip[s] = eff;
    }
    return 0;
}

/* Backward pass of the training loss
 *   L = (1/n) sum_s ((softplus(o_s) - t_s) * inv_scale)^2
 * with respect to all parameters (mean/inv_std excluded: fixed).  The bf16
 * rounding of GEMM operands uses the straight-through gradient: forward uses
 * the rounded operands, backward treats the rounding as identity but
 * multiplies by the rounded partner operand, as the GPU's GEMMs do.
 * grad[ORC_MLP_NPARAM] receives dL/dparam (zeros for mean/inv_std).
 * Returns L through loss_out. */
int orc_mlp_backward(const double *P, int64_t n, const double *raw, const double *target,
                     double inv_scale, double *grad, double *loss_out)
{
    memset(grad, 0, sizeof(double) * ORC_MLP_NPARAM);
    double loss = 0.0;
    for (int64_t s = 0; s < n; ++s) {
        double x[ORC_MLP_IN], z1[ORC_MLP_H], h1[ORC_MLP_H], z2[ORC_MLP_H], h2[ORC_MLP_H];
        mlp_features(P, raw + ORC_MLP_IN * s, x);
        double o = mlp_forward(P, x, z1, h1, z2, h2);
        double r = (softplus(o) - target[s]) * inv_scale;
        loss += r * r;
        /* dL/do for this sample */
        double go = 2.0 * r * inv_scale * sigmoid(o) / (double)n;
        /* layer 3: o = sum_k bf(w3_k) bf(h2_k) + b3 */
        double gh2[ORC_MLP_H];
        grad[ORC_MLP_OFF_B3] += go;
        for (int k = 0; k < ORC_MLP_H; ++k) {
            grad[ORC_MLP_OFF_W3 + k] += go * to_bf16(h2[k]);
            gh2[k] = go * to_bf16(P[ORC_MLP_OFF_W3 + k]);
        }
        /* layer 2 */
        double gz2[ORC_MLP_H], gh1[ORC_MLP_H];
        for (int j = 0; j < ORC_MLP_H; ++j) gz2[j] = gh2[j] * gelu_grad(z2[j]);
        for (int k = 0; k < ORC_MLP_H; ++k) gh1[k] = 0.0;
        for (int j = 0; j < ORC_MLP_H; ++j) {
            grad[ORC_MLP_OFF_B2 + j] += gz2[j];
            for (int k = 0; k < ORC_MLP_H; ++k) {
                grad[ORC_MLP_OFF_W2 + j * ORC_MLP_H + k] += gz2[j] * to_bf16(h1[k]);
                gh1[k] += gz2[j] * to_bf16(P[ORC_MLP_OFF_W2 + j * ORC_MLP_H + k]);
            }
        }
        /* layer 1 */
        for (int j = 0; j < ORC_MLP_H; ++j) {
            double gz1 = gh1[j] * gelu_grad(z1[j]);
            grad[ORC_MLP_OFF_B1 + j] += gz1;
            for (int k = 0; k < ORC_MLP_IN; ++k)
                grad[ORC_MLP_OFF_W1 + j * ORC_MLP_IN + k] += gz1 * to_bf16(x[k]);
        }
    }
    if (loss_out) *loss_out = loss / (double)n;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Single-cell collision                                                     */
/* ------------------------------------------------------------------------ */
typedef struct {
    lattice L;
    mrt_basis B;
    int have_mrt;
} ctx_t;

static int make_ctx(const orc_params *p, ctx_t *cx)
{
    if (make_lattice(p->q, &cx->L)) return -1;
    if (p->collision == 4 && p->q != 27) return -1; /* the cumulant collision needs all 27 central moments */
    cx->have_mrt = 0;
    if (p->collision == 2 || p->collision == 3) {
        if (make_mrt(&cx->L, &cx->B)) return -1;
        cx->have_mrt = 1;
    }
    return 0;
}

/* Deviation of the second-order equilibrium: f_eq_i - w_i with
 * f_eq_i = w_i rho (1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u), written so that no
 * O(1) term is formed: w_i (drho + rho (3 c.u + 9/2 (c.u)^2 - 3/2 u.u)). */
static void deq(const lattice *L, double drho, const double u[3], double *out)
{
    double rho = 1.0 + drho;
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    for (int i = 0; i < L->q; ++i) {
        double cu = L->c[i][0] * u[0] + L->c[i][1] * u[1] + L->c[i][2] * u[2];
        out[i] = L->w[i] * (drho + rho * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu));
    }
}

/* Guo forcing term F_i = w_i [3 (c_i - u) + 9 (c_i.u) c_i] . F */
static void guo(const lattice *L, const double u[3], const double F[3], double *out)
{
    for (int i = 0; i < L->q; ++i) {
        double cu = L->c[i][0] * u[0] + L->c[i][1] * u[1] + L->c[i][2] * u[2];
        double s = 0.0;
        for (int a = 0; a < 3; ++a) s += (3.0 * (L->c[i][a] - u[a]) + 9.0 * cu * L->c[i][a]) * F[a];
        out[i] = L->w[i] * s;
    }
}

/* Non-equilibrium stress Pi_ab = sum_i c_ia c_ib (d_i - deq_i), in the order
 * xx, yy, zz, xy, xz, yz. */
static void pi_neq(const lattice *L, const double *d, const double *de, double P[6])
{
    for (int k = 0; k < 6; ++k) P[k] = 0.0;
    for (int i = 0; i < L->q; ++i) {
        double n = d[i] - de[i];
        const int *c = L->c[i];
        P[0] += c[0] * c[0] * n;
        P[1] += c[1] * c[1] * n;
        P[2] += c[2] * c[2] * n;
        P[3] += c[0] * c[1] * n;
        P[4] += c[0] * c[2] * n;
        P[5] += c[1] * c[2] * n;
    }
}

/* Smagorinsky relaxation time (Yu 2005 form): with nu_t = (C_s)^2 |S|,
 * |S| = sqrt(2 S:S) and Pi_neq = -2 rho c_s^2 tau S, tau solves
 * tau^2 - tau0 tau - (9 sqrt2 / 2) C_s^2 sqrt(Q) / rho = 0, Q = Pi:Pi. */
static double tau_smag(double tau0, double cs, const double P[6], double rho)
{
    double Q = P[0] * P[0] + P[1] * P[1] + P[2] * P[2] + 2.0 * (P[3] * P[3] + P[4] * P[4] + P[5] * P[5]);
    return 0.5 * (tau0 + sqrt(tau0 * tau0 + 18.0 * sqrt(2.0) * cs * cs * sqrt(Q) / rho));
}

/* E[X_k1 X_k2 ... X_kn] of a zero-mean Gaussian with covariance S: the sum
 * over all pairings of the indices of the products of the paired
 * covariances (Isserlis), by recursion on the first index. */
static double gauss_moment(const double S[3][3], const int *idx, int n)
{
    if (n == 0) return 1.0;
    if (n % 2) return 0.0;
    double sum = 0.0;
    int rest[8];
    for (int j = 1; j < n; ++j) {
        int k = 0;
        for (int t = 1; t < n; ++t)
            if (t != j) rest[k++] = idx[t];
        sum += S[idx[0]][idx[j]] * gauss_moment(S, rest, n - 2);
    }
    return sum;
}

/* Cumulant collision (Sec. 5.1.1: cumulants instead of moments relaxed to
 * their equilibria, Geier et al. 2015), D3Q27, in the form with every
 * cumulant of order >= 3 relaxed at rate 1 (to zero):
 *   - u = (j + F/2)/rho; the second-order cumulants are the covariance
 *     S = sum f (c - u)(c - u) / rho;
 *   - the deviatoric part of S relaxes at 1/tau, its trace at omega_bulk
 *     towards 3 c_s^2 = 1;
 *   - the post-collision distribution has density rho, first-order central
 *     moments F/2 (the force enters through the velocity shift and these,
 *     so that sum c f* = j + F), second-order central moments rho S*, and
 *     higher central moments rho E[X^a Y^b Z^c] of a zero-mean Gaussian with
 *     covariance S* (all higher cumulants zero);
 *   - the populations follow from the q central moments by solving the
 *     linear system V f* = kappa*, V_(abc),i = (c_i - u)^(a,b,c), a,b,c <= 2. */
static void cumulant_cell(const orc_params *p, const lattice *L, const double *d, double tau, double rho,
                          const double u[3], double *dout)
{
    int q = L->q;
    double f[OQ], S[3][3];
    for (int i = 0; i < q; ++i) f[i] = L->w[i] + d[i];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double k2 = 0.0;
            for (int i = 0; i < q; ++i) k2 += f[i] * (L->c[i][a] - u[a]) * (L->c[i][b] - u[b]);
            S[a][b] = k2 / rho;
        }
    double om = 1.0 / tau, ob = p->omega_bulk;
    double tr = S[0][0] + S[1][1] + S[2][2];
    double Sp[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double dev = S[a][b] - (a == b ? tr / 3.0 : 0.0);
            Sp[a][b] = (1.0 - om) * dev + (a == b ? (tr - ob * (tr - 1.0)) / 3.0 : 0.0);
        }
    /* rows (a, b, c) with a, b, c <= 2 in the order a + 3 b + 9 c */
    double V[OQ][OQ], Vinv[OQ][OQ], kap[OQ];
    for (int r = 0; r < 27; ++r) {
        int e[3] = {r % 3, (r / 3) % 3, r / 9};
        for (int i = 0; i < q; ++i) {
            double v = 1.0;
            for (int a = 0; a < 3; ++a)
                for (int k = 0; k < e[a]; ++k) v *= L->c[i][a] - u[a];
            V[r][i] = v;
        }
        int order = e[0] + e[1] + e[2];
        if (order == 0) kap[r] = rho;
        else if (order == 1) kap[r] = 0.5 * p->force[e[0] ? 0 : (e[1] ? 1 : 2)];
        else {
            int idx[6], n = 0;
            for (int a = 0; a < 3; ++a)
                for (int k = 0; k < e[a]; ++k) idx[n++] = a;
            kap[r] = rho * gauss_moment(Sp, idx, n);
        }
    }
    invert(q, V, Vinv);
    for (int i = 0; i < q; ++i) {
        double fi = 0.0;
        for (int r = 0; r < q; ++r) fi += Vinv[i][r] * kap[r];
        dout[i] = fi - L->w[i];
    }
}

/* Collide one cell: d_in -> d_out (deviations).  Also returns rho, u (Guo
 * velocity) and the relaxation time used. */
static void collide_cell(const orc_params *p, const ctx_t *cx, const double *d, double *dout,
                         double *rho_out, double u[3], double *tau_out)
{
    const lattice *L = &cx->L;
    int q = L->q;
    double drho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < q; ++i) {
        drho += d[i];
        for (int a = 0; a < 3; ++a) j[a] += L->c[i][a] * d[i];
    }
    double rho = 1.0 + drho;
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * p->force[a]) / rho;
    double de[OQ], Fi[OQ];
    deq(L, drho, u, de);
    guo(L, u, p->force, Fi);

    double tau = p->tau;
    if (p->closure == 1 || p->closure == 2) {
        double P[6];
        pi_neq(L, d, de, P);
        double ts = tau_smag(p->tau, p->cs_smag, P, rho);
        tau = ts;
        if (p->closure == 2 && p->mlp) {
            double raw[ORC_MLP_IN] = {P[0], P[1], P[2], P[3], P[4], P[5], drho};
            double x[ORC_MLP_IN];
            int bad = mlp_features(p->mlp, raw, x);
            double o = mlp_forward(p->mlp, x, NULL, NULL, NULL, NULL);
            if (!bad && isfinite(o)) tau = p->tau + softplus(o);
        }
    }
    *tau_out = tau;
    *rho_out = rho;

    if (p->collision == 4) { /* cumulant (D3Q27) */
        cumulant_cell(p, L, d, tau, rho, u, dout);
    } else if (p->collision == 0) { /* SRT */
        double om = 1.0 / tau;
        for (int i = 0; i < q; ++i) dout[i] = d[i] - om * (d[i] - de[i]) + (1.0 - 0.5 * om) * Fi[i];
    } else if (p->collision == 1) { /* TRT */
        double omp = 1.0 / tau;
        double taum = 0.5 + p->magic / (tau - 0.5);
        double omm = 1.0 / taum;
        for (int i = 0; i < q; ++i) {
            int o = L->opp[i];
            double dp = 0.5 * (d[i] + d[o]), dm = 0.5 * (d[i] - d[o]);
            double ep = 0.5 * (de[i] + de[o]), em = 0.5 * (de[i] - de[o]);
            double fp = 0.5 * (Fi[i] + Fi[o]), fm = 0.5 * (Fi[i] - Fi[o]);
            dout[i] = d[i] - omp * (dp - ep) - omm * (dm - em) + (1.0 - 0.5 * omp) * fp + (1.0 - 0.5 * omm) * fm;
        }
    } else { /* MRT, Eq. 3 plus the Guo source M^{-1} (I - S/2) M F */
        const mrt_basis *B = &cx->B;
        double s[OQ];
        for (int r = 0; r < q; ++r) {
            switch (B->kind[r]) {
            case 0: s[r] = 0.0; break;
            case 1: s[r] = 1.0 / tau; break;
            case 2: s[r] = p->omega_bulk; break;
            default: s[r] = p->omega_higher; break;
            }
        }
        if (p->collision == 3) {
            /* KBC entropic stabilisation (Sec. 5.1.1; Boesch, Chikatamarla,
             * Karlin 2015): split f - f_eq by moment class into the kinematic
             * part k (conserved moments), the shear part s (deviatoric second
             * moments) and the rest h (trace of the second moments and all
             * higher moments).  s relaxes at 2 beta = 1/tau; h at gamma beta,
             * with gamma the stationary point of the quadratic entropy
             * sum (f* - f_eq)^2 / f_eq of the post-collision state:
             * gamma = 1/beta - (2 - 1/beta) <ds|dh> / <dh|dh>,
             * <x|y> = sum x_i y_i / f_eq_i; gamma = 2 when dh vanishes. */
            double mneq[OQ], ds[OQ], dh[OQ];
            for (int r = 0; r < q; ++r) {
                mneq[r] = 0.0;
                for (int i = 0; i < q; ++i) mneq[r] += B->M[r][i] * (d[i] - de[i]);
            }
            for (int i = 0; i < q; ++i) {
                ds[i] = dh[i] = 0.0;
                for (int r = 0; r < q; ++r) {
                    if (B->kind[r] == 1) ds[i] += B->Minv[i][r] * mneq[r];
                    else if (B->kind[r] >= 2) dh[i] += B->Minv[i][r] * mneq[r];
                }
            }
            double sh = 0.0, hh = 0.0;
            for (int i = 0; i < q; ++i) {
                double feq = L->w[i] + de[i];
                sh += ds[i] * dh[i] / feq;
                hh += dh[i] * dh[i] / feq;
            }
            double beta = 0.5 / tau;
            double gamma = hh > 1e-30 ? 1.0 / beta - (2.0 - 1.0 / beta) * sh / hh : 2.0;
            for (int r = 0; r < q; ++r)
                if (B->kind[r] >= 2) s[r] = gamma * beta;
        }
        double g[OQ];
        for (int r = 0; r < q; ++r) {
            double mneq = 0.0, mf = 0.0;
            for (int i = 0; i < q; ++i) {
                mneq += B->M[r][i] * (d[i] - de[i]);
                mf += B->M[r][i] * Fi[i];
            }
            g[r] = s[r] * mneq - (1.0 - 0.5 * s[r]) * mf;
        }
        for (int i = 0; i < q; ++i) {
            double corr = 0.0;
            for (int r = 0; r < q; ++r) corr += B->Minv[i][r] * g[r];
            dout[i] = d[i] - corr;
        }
    }
}

/* Public single-cell entry for unit tests.  rho_u_tau[5] = rho, u, tau. */
int orc_collide_cell(const orc_params *p, const double *d, double *dout, double *rho_u_tau)
{
    ctx_t cx;
    if (make_ctx(p, &cx)) return -1;
    double rho, u[3], tau;
    collide_cell(p, &cx, d, dout, &rho, u, &tau);
    rho_u_tau[0] = rho;
    rho_u_tau[1] = u[0];
    rho_u_tau[2] = u[1];
    rho_u_tau[3] = u[2];
    rho_u_tau[4] = tau;
    return 0;
}

/* Equilibrium deviations for given rho, u (one cell). */
int orc_equilibrium(int q, double rho, const double *u, double *out)
{
    lattice L;
    if (make_lattice(q, &L)) return -1;
    deq(&L, rho - 1.0, u, out);
    return 0;
}

/* Guo forcing term (one cell). */
int orc_guo(int q, const double *u, const double *F, double *out)
{
    lattice L;
    if (make_lattice(q, &L)) return -1;
    guo(&L, u, F, out);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Global lattice: initialisation, collision, pull streaming, moments        */
/* ------------------------------------------------------------------------ */
static inline int64_t lin(int x, int y, int z, int nx, int ny) { return ((int64_t)z * ny + y) * nx + x; }

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* d[q][N] = f_eq(rho, u) - w for fluid cells, 0 for solid cells.
 * rho[N], u[3][N] in global x-fastest order. */
int orc_init(int q, int nx, int ny, int nz, const double *rho, const double *u, const uint8_t *solid, double *d)
{
    lattice L;
    if (make_lattice(q, &L)) return -1;
    int64_t N = (int64_t)nx * ny * nz;
    for (int64_t n = 0; n < N; ++n) {
        double de[OQ];
        if (solid && solid[n]) {
            for (int i = 0; i < q; ++i) d[i * N + n] = 0.0;
            continue;
        }
        double uu[3] = {u[n], u[N + n], u[2 * N + n]};
        deq(&L, rho[n] - 1.0, uu, de);
        for (int i = 0; i < q; ++i) d[i * N + n] = de[i];
    }
    return 0;
}

/* Collision over all fluid cells: post[q][N], uvel[3][N] (collision-time u). */
static void collide_all(const orc_params *p, const ctx_t *cx, int nx, int ny, int nz,
                        const uint8_t *solid, const double *d, double *post, double *uvel)
{
    int q = cx->L.q;
    int64_t N = (int64_t)nx * ny * nz;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int64_t n = lin(x, y, z, nx, ny);
                if (solid && solid[n]) {
                    for (int i = 0; i < q; ++i) post[i * N + n] = 0.0;
                    uvel[n] = uvel[N + n] = uvel[2 * N + n] = 0.0;
                    continue;
                }
                double dc[OQ], dp[OQ], rho, u[3], tau;
                for (int i = 0; i < q; ++i) dc[i] = d[i * N + n];
                collide_cell(p, cx, dc, dp, &rho, u, &tau);
                for (int i = 0; i < q; ++i) post[i * N + n] = dp[i];
                uvel[n] = u[0];
                uvel[N + n] = u[1];
                uvel[2 * N + n] = u[2];
            }
}

/* Pull streaming with boundaries.  For fluid x and direction i the source is
 * s = x - c_i (wrapped on periodic axes):
 *   s beyond a wall (non-periodic axis that is not the pressure axis), or s
 *   solid: half-way bounce-back, d_i(x) = post_opp(i)(x);
 *   s beyond the pressure faces: anti-bounce-back with the wall density and
 *   the cell's own collision-time velocity;
 *   otherwise d_i(x) = post_i(s). */
static void stream_all(const orc_params *p, const lattice *L, int nx, int ny, int nz,
                       const uint8_t *solid, const double *post, const double *uvel, double *dnew)
{
    int q = L->q;
    int64_t N = (int64_t)nx * ny * nz;
    int ext[3] = {nx, ny, nz};
#pragma omp parallel for schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int64_t n = lin(x, y, z, nx, ny);
                if (solid && solid[n]) {
                    for (int i = 0; i < q; ++i) dnew[i * N + n] = 0.0;
                    continue;
                }
                int pos[3] = {x, y, z};
                for (int i = 0; i < q; ++i) {
                    int s[3], wall = 0, press = 0;
                    double rho_w = 1.0;
                    for (int a = 0; a < 3; ++a) {
                        s[a] = pos[a] - L->c[i][a];
                        if (s[a] < 0 || s[a] >= ext[a]) {
                            if (p->periodic[a]) {
                                s[a] = (s[a] + ext[a]) % ext[a];
                            } else if (a == p->pressure_axis) {
                                press = 1;
                                rho_w = (s[a] < 0) ? p->rho_in : p->rho_out;
                            } else {
                                wall = 1;
                            }
                        }
                    }
                    int io = L->opp[i];
                    if (wall) {
                        dnew[i * N + n] = post[io * N + n];
                    } else if (press) {
                        double u[3] = {uvel[n], uvel[N + n], uvel[2 * N + n]};
                        double cu = L->c[i][0] * u[0] + L->c[i][1] * u[1] + L->c[i][2] * u[2];
                        double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
                        /* f_i = -f*_opp + 2 w rho_w (1 + 9/2 (c.u)^2 - 3/2 u.u), in deviations */
                        dnew[i * N + n] = -post[io * N + n]
                                          + 2.0 * L->w[i] * (rho_w * (1.0 + 4.5 * cu * cu - 1.5 * uu) - 1.0);
                    } else {
                        int64_t m = lin(s[0], s[1], s[2], nx, ny);
                        if (solid && solid[m]) dnew[i * N + n] = post[io * N + n];
                        else dnew[i * N + n] = post[i * N + m];
                    }
                }
            }
}

/* Streaming only (no collision): d_new from post.  uvel may be NULL when no
 * pressure boundary is used. */
int orc_stream(const orc_params *p, int nx, int ny, int nz, const uint8_t *solid, const double *post,
               const double *uvel, double *dnew)
{
    lattice L;
    if (make_lattice(p->q, &L)) return -1;
    if (p->pressure_axis >= 0 && !uvel) return -2;
    stream_all(p, &L, nx, ny, nz, solid, post, uvel, dnew);
    return 0;
}

/* Collision only over the lattice: post[q][N] and uvel[3][N]. */
int orc_collide(const orc_params *p, int nx, int ny, int nz, const uint8_t *solid, const double *d,
                double *post, double *uvel, int nthreads)
{
    ctx_t cx;
    if (make_ctx(p, &cx)) return -1;
    set_threads(nthreads);
    collide_all(p, &cx, nx, ny, nz, solid, d, post, uvel);
    return 0;
}

/* nsteps full updates (Eq. 2) of d[q][N] in place.  Scratch is allocated
 * here.  nthreads <= 0 keeps the OpenMP default. */
int orc_run(const orc_params *p, int nx, int ny, int nz, const uint8_t *solid, double *d, int nsteps,
            int nthreads)
{
    ctx_t cx;
    if (make_ctx(p, &cx)) return -1;
    if (!(p->tau > 0.5)) return -3;
    set_threads(nthreads);
    int q = p->q;
    int64_t N = (int64_t)nx * ny * nz;
    double *post = (double *)malloc(sizeof(double) * q * N);
    double *uvel = (double *)malloc(sizeof(double) * 3 * N);
    if (!post || !uvel) {
        free(post);
        free(uvel);
        return -4;
    }
    for (int t = 0; t < nsteps; ++t) {
        collide_all(p, &cx, nx, ny, nz, solid, d, post, uvel);
        stream_all(p, &cx.L, nx, ny, nz, solid, post, uvel, d);
    }
    free(post);
    free(uvel);
    return 0;
}

/* Kahan-compensated accumulator */
typedef struct { double s, c; } kahan;
static void kadd(kahan *k, double v)
{
    double y = v - k->c;
    double t = k->s + y;
    k->c = (t - k->s) - y;
    k->s = t;
}

/* Moments (Eq. 1) of the state d: rho[N], u[3][N] with u = (j + F/2)/rho;
 * solid cells get rho = 0, u = 0.  totals[8] = mass, momentum x/y/z (sum of
 * rho u), kinetic energy sum rho |u|^2 / 2, max |u|, number of fluid cells,
 * 0.  Any output pointer may be NULL. */
int orc_moments(int q, const double *force, int nx, int ny, int nz, const uint8_t *solid, const double *d,
                double *rho_out, double *u_out, double *totals)
{
    lattice L;
    if (make_lattice(q, &L)) return -1;
    int64_t N = (int64_t)nx * ny * nz;
    kahan km = {0, 0}, kx = {0, 0}, ky = {0, 0}, kz = {0, 0}, ke = {0, 0};
    double umax = 0.0, nfl = 0.0;
    for (int64_t n = 0; n < N; ++n) {
        if (solid && solid[n]) {
            if (rho_out) rho_out[n] = 0.0;
            if (u_out) u_out[n] = u_out[N + n] = u_out[2 * N + n] = 0.0;
            continue;
        }
        double drho = 0.0, j[3] = {0, 0, 0};
        for (int i = 0; i < q; ++i) {
            double v = d[i * N + n];
            drho += v;
            for (int a = 0; a < 3; ++a) j[a] += L.c[i][a] * v;
        }
        double rho = 1.0 + drho, u[3];
        for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * force[a]) / rho;
        if (rho_out) rho_out[n] = rho;
        if (u_out) {
            u_out[n] = u[0];
            u_out[N + n] = u[1];
            u_out[2 * N + n] = u[2];
        }
        double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        kadd(&km, rho);
        kadd(&kx, rho * u[0]);
        kadd(&ky, rho * u[1]);
        kadd(&kz, rho * u[2]);
        kadd(&ke, 0.5 * rho * uu);
        if (sqrt(uu) > umax) umax = sqrt(uu);
        nfl += 1.0;
    }
    if (totals) {
        totals[0] = km.s;
        totals[1] = kx.s;
        totals[2] = ky.s;
        totals[3] = kz.s;
        totals[4] = ke.s;
        totals[5] = umax;
        totals[6] = nfl;
        totals[7] = 0.0;
    }
    return 0;
}

/* Momentum exchange (Sec. "Geometrically fully resolved simulations": the
 * force on an obstacle is the momentum that the bounced-back populations
 * hand to it, after Ladd 1994 / Aidun 1998).  With half-way bounce-back on a
 * resting obstacle, the post-collision population f*_j(x) of a fluid cell x
 * whose target x + c_j is a solid cell or lies beyond a wall comes back to x
 * as f_opp(j)(x) = f*_j(x): the obstacle receives c_j f*_j on the way in and
 * again on the way out, 2 c_j f*_j per such link and step.  Links across the
 * pressure faces (anti-bounce-back) are not obstacles and are not counted;
 * a link leaving through a wall and a pressure face at once counts as a wall
 * link, as in the streaming above.
 * post: the step's post-collision deviations (orc_collide), so
 * f*_j = w_j + post_j.  out[8]: force on the solid cells (x, y, z), force on
 * the walls (x, y, z), number of solid links, number of wall links.  Serial,
 * Kahan-compensated sums. */
int orc_momentum_exchange(const orc_params *p, int nx, int ny, int nz, const uint8_t *solid, const double *post,
                          double *out)
{
    lattice L;
    if (make_lattice(p->q, &L)) return -1;
    int q = L.q;
    int64_t N = (int64_t)nx * ny * nz;
    int ext[3] = {nx, ny, nz};
    kahan fs[3] = {{0, 0}, {0, 0}, {0, 0}}, fw[3] = {{0, 0}, {0, 0}, {0, 0}};
    double ns = 0.0, nw = 0.0;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int64_t n = lin(x, y, z, nx, ny);
                if (solid && solid[n]) continue;
                int pos[3] = {x, y, z};
                for (int j = 0; j < q; ++j) {
                    int t[3], wall = 0, press = 0;
                    for (int a = 0; a < 3; ++a) {
                        t[a] = pos[a] + L.c[j][a];
                        if (t[a] < 0 || t[a] >= ext[a]) {
                            if (p->periodic[a]) t[a] = (t[a] + ext[a]) % ext[a];
                            else if (a == p->pressure_axis) press = 1;
                            else wall = 1;
                        }
                    }
                    int to_solid = 0;
                    if (!wall && !press && solid) to_solid = solid[lin(t[0], t[1], t[2], nx, ny)] != 0;
                    if (!wall && !to_solid) continue;
                    double f = L.w[j] + post[j * N + n];
                    for (int a = 0; a < 3; ++a) kadd(wall ? &fw[a] : &fs[a], 2.0 * L.c[j][a] * f);
                    if (wall) nw += 1.0;
                    else ns += 1.0;
                }
            }
    for (int a = 0; a < 3; ++a) {
        out[a] = fs[a].s;
        out[3 + a] = fw[a].s;
    }
    out[6] = ns;
    out[7] = nw;
    return 0;
}

int orc_mlp_nparam(void) { return ORC_MLP_NPARAM; }
