/*
 * z4c_oracle.c -- plain, slow, FP64 reference of the vacuum Z4c evolution
 * step.  TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark are the only callers.  It shares no code,
 * header or constant table with the HIP library; it is written straight from
 * the equations, one grid point at a time, with full 3x3 index loops.
 *
 * What it computes (paper: "SACRA-K", arXiv 2607.08743):
 *   - evolved variables W, gt_ij, Khat, At_ij, Gt^i, Theta, alpha, beta^i, B^i
 *     (Sec. 2.1.1, conformal-variable definitions and the gauge equations);
 *   - the Z4c right-hand side in the W form of the Z4c literature the paper
 *     cites in Sec. 2.1.1 (Bernuzzi & Hilditch 2010; Hilditch et al. 2013),
 *     with constraint damping kappa1, kappa2 (and kappa3, default 0);
 *   - 1+log slicing and the Gamma-driver shift with coefficient 0.75 and
 *     damping eta (Sec. 2.1.1, gauge equations);
 *   - 4th-order centred first/second differences, 4th-order upwinded shift
 *     advection biased by the sign of the shift, 6th-order Kreiss-Oliger
 *     dissipation with sigma = 0.5 (Sec. 2.2, spatial discretisation);
 *   - classical RK4 in method-of-lines form (Sec. 2.2);
 *   - the Sommerfeld outgoing condition on the outer boundary (Sec. 2.2.2);
 *   - enforcement of det gt = 1 and tr At = 0 (Sec. 2.1.1 states both hold
 *     by construction; how they are restored is a reading, see below).
 *
 * Readings where the paper is silent (each also listed in the design notes):
 *   - K in the 1+log condition is Khat unless lapse_uses_K = 1 (then Khat+2Theta);
 *   - the mixed derivative is the tensor product D1_a(D1_b f), a < b;
 *   - the upwind stencil is the 5-point lopsided one, shifted toward +s with
 *     s = +1 when beta^d >= 0;
 *   - KO acts on all 25 fields at active points, +sigma/(64 h) * delta^6;
 *   - outer-boundary ghost points of a Sommerfeld box are evolved with
 *     -(x^i/r) d_i f - (f - f_flat)/r, 2nd-order differences (one-sided at
 *     the array edge), speed 1 for every field;
 *   - enforcement: gt <- gt / cbrt(det gt), then At <- At - gt (gu.At)/3 with
 *     gu the inverse of the rescaled gt;
 *   - 1/W in the Gt equation uses max(W, w_floor);
 *   - equatorial symmetry (Sec. 2.2.2 / Sec. 2.4 use it to halve the work):
 *     the lower z face of the active box is the plane z = 0; ghost layer
 *     k = ng-1-m holds the value of layer ng+m times (-1)^(number of z
 *     indices of the component), for every i, j; the other five faces are
 *     Sommerfeld faces as above.
 *
 * Data layout (numpy order [f][k][j][i], x fastest):
 *   u[f*sf + (k*Ny + j)*Nx + i], Nx = nx + 2 ng, ..., i in [0, Nx).
 *   Active cells are i in [ng, ng+nx); cell centre x = x0 + (i - ng) * dx.
 *
 * Compile: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp (no FMA
 * contraction, so the pi-mirror pairs round identically).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NF 25

/* field indices */
enum {
    IW = 0, IGT = 1, /* gt_xx gt_xy gt_xz gt_yy gt_yz gt_zz : 1..6 */
    IKH = 7, IAT = 8, /* At_xx .. At_zz : 8..13 */
    IGAM = 14,        /* Gt^x Gt^y Gt^z : 14..16 */
    ITH = 17, IAL = 18, IBE = 19, /* beta^x..z : 19..21 */
    IBB = 22          /* B^x..z : 22..24 */
};

enum { BC_PERIODIC = 0, BC_SOMMERFELD = 1, BC_COPY = 2, BC_EQUATORIAL = 3 };

typedef struct {
    double kappa1, kappa2, kappa3, eta, shift_coeff, ko_sigma, w_floor;
    int lapse_uses_K;
} oz_params;

typedef struct {
    int n[3];     /* active cells per direction */
    int ng;       /* ghost width */
    int N[3];     /* stored points per direction */
    long sf;      /* stride between fields */
    double h[3];  /* spacing */
    double x0[3]; /* centre of the first active cell */
    int bc;
} grid;

static int make_grid(grid* g, long sf, int nx, int ny, int nz, int ng, double dx, double dy, double dz,
                     double x0, double y0, double z0, int bc);

/* storage slot of the symmetric pair (a,b) inside gt_ij / At_ij */
static const int sym[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};

/* value at infinity (flat space) of every field */
static double flat_value(int f)
{
    if (f == IW || f == IAL) return 1.0;
    if (f == IGT + 0 || f == IGT + 3 || f == IGT + 5) return 1.0;
    return 0.0;
}

/* sign of field f under the reflection z -> -z: (-1)^(number of z indices) */
static double z_parity(int f)
{
    static const int tensor_z[6] = {0, 0, 1, 0, 1, 2}; /* xx xy xz yy yz zz */
    int nz = 0;
    if (f >= IGT && f < IGT + 6) nz = tensor_z[f - IGT];
    if (f >= IAT && f < IAT + 6) nz = tensor_z[f - IAT];
    if (f == IGAM + 2 || f == IBE + 2 || f == IBB + 2) nz = 1;
    return (nz % 2) ? -1.0 : 1.0;
}

static long lin(const grid* g, int i, int j, int k)
{
    return ((long)k * g->N[1] + j) * g->N[0] + i;
}

/* f at the point P shifted by s cells along direction d */
static double fv(const double* u, const grid* g, int f, const int P[3], int d, int s)
{
    int Q[3] = {P[0], P[1], P[2]};
    Q[d] += s;
    return u[f * g->sf + lin(g, Q[0], Q[1], Q[2])];
}

/* ------------------------------------------------------------------ */
/* Stencils (Sec. 2.2).  Every difference is taken from the centre    */
/* value first, so constant data gives exactly zero and mirror pairs  */
/* of points produce exactly mirrored results.                        */
/* ------------------------------------------------------------------ */

/* 4th-order centred first derivative */
static double D1(const double* u, const grid* g, int f, const int P[3], int d)
{
    double p1 = fv(u, g, f, P, d, 1), m1 = fv(u, g, f, P, d, -1);
    double p2 = fv(u, g, f, P, d, 2), m2 = fv(u, g, f, P, d, -2);
    return (8.0 * (p1 - m1) - (p2 - m2)) / (12.0 * g->h[d]);
}

/* 4th-order centred second derivative along one direction */
static double D2(const double* u, const grid* g, int f, const int P[3], int d)
{
    double c = fv(u, g, f, P, d, 0);
    double p1 = fv(u, g, f, P, d, 1), m1 = fv(u, g, f, P, d, -1);
    double p2 = fv(u, g, f, P, d, 2), m2 = fv(u, g, f, P, d, -2);
    return (16.0 * ((p1 - c) + (m1 - c)) - ((p2 - c) + (m2 - c))) / (12.0 * g->h[d] * g->h[d]);
}

/* mixed second derivative d_a d_b f (a != b) as D1_lo( D1_hi f ) */
static double DMIX(const double* u, const grid* g, int f, const int P[3], int a, int b)
{
    int lo = a < b ? a : b, hi = a < b ? b : a;
    double v[5];
    for (int s = -2; s <= 2; ++s) {
        if (s == 0) continue;
        int Q[3] = {P[0], P[1], P[2]};
        Q[lo] += s;
        v[s + 2] = D1(u, g, f, Q, hi);
    }
    return (8.0 * (v[3] - v[1]) - (v[4] - v[0])) / (12.0 * g->h[lo]);
}

static double DD(const double* u, const grid* g, int f, const int P[3], int a, int b)
{
    return a == b ? D2(u, g, f, P, a) : DMIX(u, g, f, P, a, b);
}

/* 4th-order upwinded first derivative; the stencil leans toward +s where
   s is the sign of the shift component (s = +1 when beta >= 0) */
static double DUP(const double* u, const grid* g, int f, const int P[3], int d, double beta)
{
    int s = beta >= 0.0 ? 1 : -1;
    double c = fv(u, g, f, P, d, 0);
    double m = fv(u, g, f, P, d, -s);
    double p1 = fv(u, g, f, P, d, s), p2 = fv(u, g, f, P, d, 2 * s), p3 = fv(u, g, f, P, d, 3 * s);
    return (double)s * (-3.0 * (m - c) + 18.0 * (p1 - c) - 6.0 * (p2 - c) + (p3 - c)) / (12.0 * g->h[d]);
}

/* 6th undivided difference (1,-6,15,-20,15,-6,1) */
static double KO6(const double* u, const grid* g, int f, const int P[3], int d)
{
    double c = fv(u, g, f, P, d, 0);
    double p1 = fv(u, g, f, P, d, 1), m1 = fv(u, g, f, P, d, -1);
    double p2 = fv(u, g, f, P, d, 2), m2 = fv(u, g, f, P, d, -2);
    double p3 = fv(u, g, f, P, d, 3), m3 = fv(u, g, f, P, d, -3);
    return ((p3 - c) + (m3 - c)) - 6.0 * ((p2 - c) + (m2 - c)) + 15.0 * ((p1 - c) + (m1 - c));
}

/* ------------------------------------------------------------------ */
/* 3x3 helpers                                                         */
/* ------------------------------------------------------------------ */
static double det3(double m[3][3])
{
    return m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1])
         - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0])
         + m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
}

/* inverse of a symmetric 3x3 matrix by cofactors */
static void inv3(double m[3][3], double out[3][3])
{
    double d = det3(m);
    out[0][0] = (m[1][1] * m[2][2] - m[1][2] * m[2][1]) / d;
    out[0][1] = (m[0][2] * m[2][1] - m[0][1] * m[2][2]) / d;
    out[0][2] = (m[0][1] * m[1][2] - m[0][2] * m[1][1]) / d;
    out[1][1] = (m[0][0] * m[2][2] - m[0][2] * m[2][0]) / d;
    out[1][2] = (m[0][2] * m[1][0] - m[0][0] * m[1][2]) / d;
    out[2][2] = (m[0][0] * m[1][1] - m[0][1] * m[1][0]) / d;
    out[1][0] = out[0][1];
    out[2][0] = out[0][2];
    out[2][1] = out[1][2];
}

/* ------------------------------------------------------------------ */
/* Z4c right-hand side at one active point                             */
/* ------------------------------------------------------------------ */
static void rhs_point(const double* u, const grid* g, const oz_params* p, int i, int j, int k,
                      double out[NF])
{
    const int P[3] = {i, j, k};
    double v[NF];
    for (int f = 0; f < NF; ++f) v[f] = u[f * g->sf + lin(g, i, j, k)];

    const double W = v[IW], Kh = v[IKH], Th = v[ITH], al = v[IAL];
    double gt[3][3], At[3][3], Gt[3], be[3], Bv[3];
    for (int a = 0; a < 3; ++a) {
        for (int b = 0; b < 3; ++b) {
            gt[a][b] = v[IGT + sym[a][b]];
            At[a][b] = v[IAT + sym[a][b]];
        }
        Gt[a] = v[IGAM + a];
        be[a] = v[IBE + a];
        Bv[a] = v[IBB + a];
    }

    /* derivatives: d[c] = d_c, dd[c][e] = d_c d_e */
    double dW[3], ddW[3][3], dKh[3], dTh[3], dal[3], ddal[3][3];
    double dgt[3][3][3], ddgt[3][3][3][3]; /* [c][e][a][b] */
    double dGt[3][3];                      /* d_c Gt^a : [c][a] */
    double dbe[3][3], ddbe[3][3][3];       /* d_c beta^a : [c][a]; d_c d_e beta^a : [c][e][a] */
    for (int c = 0; c < 3; ++c) {
        dW[c] = D1(u, g, IW, P, c);
        dKh[c] = D1(u, g, IKH, P, c);
        dTh[c] = D1(u, g, ITH, P, c);
        dal[c] = D1(u, g, IAL, P, c);
        for (int a = 0; a < 3; ++a) {
            dGt[c][a] = D1(u, g, IGAM + a, P, c);
            dbe[c][a] = D1(u, g, IBE + a, P, c);
            for (int b = 0; b < 3; ++b) dgt[c][a][b] = D1(u, g, IGT + sym[a][b], P, c);
        }
        for (int e = 0; e < 3; ++e) {
            ddW[c][e] = DD(u, g, IW, P, c, e);
            ddal[c][e] = DD(u, g, IAL, P, c, e);
            for (int a = 0; a < 3; ++a) {
                ddbe[c][e][a] = DD(u, g, IBE + a, P, c, e);
                for (int b = 0; b < 3; ++b) ddgt[c][e][a][b] = DD(u, g, IGT + sym[a][b], P, c, e);
            }
        }
    }

    /* inverse conformal metric */
    double gu[3][3];
    inv3(gt, gu);

    /* Christoffel symbols of gt: first kind Chr1[k][i][j] = Gamma_kij, second kind Chr2[k][i][j] */
    double Chr1[3][3][3], Chr2[3][3][3], Gtd[3];
    for (int kk = 0; kk < 3; ++kk)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                Chr1[kk][a][b] = 0.5 * (dgt[a][kk][b] + dgt[b][kk][a] - dgt[kk][a][b]);
    for (int kk = 0; kk < 3; ++kk)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double s = 0.0;
                for (int l = 0; l < 3; ++l) s += gu[kk][l] * Chr1[l][a][b];
                Chr2[kk][a][b] = s;
            }
    for (int kk = 0; kk < 3; ++kk) {
        double s = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) s += gu[a][b] * Chr2[kk][a][b];
        Gtd[kk] = s;
    }

    double Zu[3];
    for (int a = 0; a < 3; ++a) Zu[a] = 0.5 * (Gt[a] - Gtd[a]);
    const double K = Kh + 2.0 * Th;
    const double divb = dbe[0][0] + dbe[1][1] + dbe[2][2];

    /* raised At: Au[i][j] = At^i_j, Auu[i][j] = At^ij, AA = At_ij At^ij */
    double Au[3][3], Auu[3][3], AA = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int c = 0; c < 3; ++c) s += gu[a][c] * At[c][b];
            Au[a][b] = s;
        }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int c = 0; c < 3; ++c) s += Au[a][c] * gu[c][b];
            Auu[a][b] = s;
        }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) AA += At[a][b] * Auu[a][b];

    /* conformal Ricci tensor Rt_ij */
    double Rt[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double t1 = 0.0, t2 = 0.0, t3 = 0.0, t4 = 0.0;
            for (int l = 0; l < 3; ++l)
                for (int m = 0; m < 3; ++m) t1 += gu[l][m] * ddgt[l][m][a][b];
            for (int c = 0; c < 3; ++c) t2 += gt[c][a] * dGt[b][c] + gt[c][b] * dGt[a][c];
            for (int c = 0; c < 3; ++c) t3 += Gtd[c] * (Chr1[a][b][c] + Chr1[b][a][c]);
            for (int l = 0; l < 3; ++l)
                for (int m = 0; m < 3; ++m)
                    for (int c = 0; c < 3; ++c)
                        t4 += gu[l][m] * (Chr2[c][l][a] * Chr1[b][c][m] + Chr2[c][l][b] * Chr1[a][c][m]
                                          + Chr2[c][a][m] * Chr1[c][l][b]);
            Rt[a][b] = -0.5 * t1 + 0.5 * t2 + 0.5 * t3 + t4;
        }

    /* conformal-factor part: W^2 R_ij written without division */
    double DDW[3][3], trDDW = 0.0, dW2 = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int c = 0; c < 3; ++c) s += Chr2[c][a][b] * dW[c];
            DDW[a][b] = ddW[a][b] - s;
        }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            trDDW += gu[a][b] * DDW[a][b];
            dW2 += gu[a][b] * dW[a] * dW[b];
        }
    double W2R[3][3], R = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            W2R[a][b] = W * W * Rt[a][b] + W * (DDW[a][b] + gt[a][b] * trDDW) - 2.0 * gt[a][b] * dW2;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) R += gu[a][b] * W2R[a][b];

    /* W^2 D_i D_j alpha (physical covariant second derivative) and its trace */
    double dWda = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) dWda += gu[a][b] * dW[a] * dal[b];
    double W2DDa[3][3], Lapa = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int c = 0; c < 3; ++c) s += Chr2[c][a][b] * dal[c];
            W2DDa[a][b] = W * W * (ddal[a][b] - s) + W * (dW[a] * dal[b] + dW[b] * dal[a] - gt[a][b] * dWda);
        }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) Lapa += gu[a][b] * W2DDa[a][b];

    /* trace-free part of W^2 (-D_i D_j alpha + alpha R_ij) */
    double X[3][3], trX = 0.0, XTF[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) X[a][b] = -W2DDa[a][b] + al * W2R[a][b];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) trX += gu[a][b] * X[a][b];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) XTF[a][b] = X[a][b] - gt[a][b] * trX / 3.0;

    /* non-advective right-hand sides N[f] */
    double N[NF];
    N[IW] = W * (al * K - divb) / 3.0;
    for (int a = 0; a < 3; ++a)
        for (int b = a; b < 3; ++b) {
            double lg = 0.0, la = 0.0, aa = 0.0;
            for (int c = 0; c < 3; ++c) {
                lg += gt[a][c] * dbe[b][c] + gt[b][c] * dbe[a][c];
                la += At[a][c] * dbe[b][c] + At[b][c] * dbe[a][c];
                aa += At[a][c] * Au[c][b];
            }
            N[IGT + sym[a][b]] = -2.0 * al * At[a][b] + lg - 2.0 * gt[a][b] * divb / 3.0;
            N[IAT + sym[a][b]] = XTF[a][b] + al * (K * At[a][b] - 2.0 * aa) + la - 2.0 * At[a][b] * divb / 3.0;
        }
    N[IKH] = -Lapa + al * (AA + K * K / 3.0) + al * p->kappa1 * (1.0 - p->kappa2) * Th;

    const double Wr = W > p->w_floor ? W : p->w_floor;
    for (int a = 0; a < 3; ++a) {
        double t_ada = 0.0, t_chr = 0.0, t_aw = 0.0, t_dk = 0.0, t_ddb = 0.0, t_ddb2 = 0.0, t_gdb = 0.0,
               t_zdb = 0.0;
        for (int b = 0; b < 3; ++b) {
            t_ada += Auu[a][b] * dal[b];
            t_aw += Auu[a][b] * dW[b];
            t_dk += gu[a][b] * (2.0 * dKh[b] + dTh[b]);
            t_gdb += Gtd[b] * dbe[b][a];
            t_zdb += Zu[b] * dbe[b][a];
            for (int c = 0; c < 3; ++c) {
                t_chr += Chr2[a][b][c] * Auu[b][c];
                t_ddb += gu[b][c] * ddbe[b][c][a];
                t_ddb2 += gu[a][b] * ddbe[b][c][c];
            }
        }
        N[IGAM + a] = -2.0 * t_ada + 2.0 * al * t_chr - 6.0 * al * t_aw / Wr - 2.0 * al * t_dk / 3.0 + t_ddb
                    + t_ddb2 / 3.0 + 2.0 * Gtd[a] * divb / 3.0 - t_gdb - 2.0 * al * p->kappa1 * Zu[a]
                    + 2.0 * p->kappa3 * (2.0 * Zu[a] * divb / 3.0 - t_zdb);
    }
    N[ITH] = 0.5 * al * (R - AA + 2.0 * K * K / 3.0) - al * p->kappa1 * (2.0 + p->kappa2) * Th;
    N[IAL] = -2.0 * al * (p->lapse_uses_K ? K : Kh);
    for (int a = 0; a < 3; ++a) {
        N[IBE + a] = p->shift_coeff * Bv[a];
        N[IBB + a] = N[IGAM + a] - p->eta * Bv[a];
    }

    /* shift advection (upwinded) and Kreiss-Oliger dissipation on every field */
    for (int f = 0; f < NF; ++f) {
        double adv = 0.0, ko = 0.0;
        for (int d = 0; d < 3; ++d) {
            adv += be[d] * DUP(u, g, f, P, d, be[d]);
            ko += p->ko_sigma / (64.0 * g->h[d]) * KO6(u, g, f, P, d);
        }
        out[f] = N[f] + adv + ko;
    }
}

/* ------------------------------------------------------------------ */
/* Constraints (Sec. 2.3, vacuum): Hamiltonian H and momentum M^i      */
/*   H   = R + K^2 - K_ij K^ij = R - At_ij At^ij + (2/3) K^2           */
/*   M^i = D_j (K^ij - gamma^ij K)                                     */
/*       = W^2 [ Dt_j At^ij - 3 At^ij d_j W / W - (2/3) gt^ij d_j K ]  */
/* with K = Khat + 2 Theta (the ADM trace), R built exactly as in the  */
/* right-hand side (evolved Gt in its d Gt term), Dt the covariant     */
/* derivative of gt: Dt_j At^ij = d_j At^ij + Chr^i_jk At^jk           */
/*                                + Chr^j_jk At^ik,                    */
/* and d_j At^ij = gu^ia gu^jb d_j At_ab + At_ab d_j(gu^ia gu^jb),     */
/* d_j gu^ia = -gu^ic gu^ad d_j gt_cd.                                 */
/* ------------------------------------------------------------------ */
static void constraints_point(const double* u, const grid* g, const oz_params* p, int i, int j, int k,
                              double out[4])
{
    (void)p;
    const int P[3] = {i, j, k};
    const long q = lin(g, i, j, k);
    const double W = u[IW * g->sf + q];
    const double K = u[IKH * g->sf + q] + 2.0 * u[ITH * g->sf + q];
    double gt[3][3], At[3][3], gu[3][3], Gt[3];
    for (int a = 0; a < 3; ++a) {
        for (int b = 0; b < 3; ++b) {
            gt[a][b] = u[(IGT + sym[a][b]) * g->sf + q];
            At[a][b] = u[(IAT + sym[a][b]) * g->sf + q];
        }
        Gt[a] = u[(IGAM + a) * g->sf + q];
    }
    inv3(gt, gu);
    double dW[3], ddW[3][3], dK[3], dgt[3][3][3], ddgt[3][3][3][3], dGt[3][3], dAt[3][3][3];
    for (int c = 0; c < 3; ++c) {
        dW[c] = D1(u, g, IW, P, c);
        dK[c] = D1(u, g, IKH, P, c) + 2.0 * D1(u, g, ITH, P, c);
        for (int a = 0; a < 3; ++a) {
            dGt[c][a] = D1(u, g, IGAM + a, P, c);
            for (int b = 0; b < 3; ++b) {
                dgt[c][a][b] = D1(u, g, IGT + sym[a][b], P, c);
                dAt[c][a][b] = D1(u, g, IAT + sym[a][b], P, c);
            }
        }
        for (int e = 0; e < 3; ++e) {
            ddW[c][e] = DD(u, g, IW, P, c, e);
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) ddgt[c][e][a][b] = DD(u, g, IGT + sym[a][b], P, c, e);
        }
    }
    double Chr1[3][3][3], Chr2[3][3][3], Gtd[3];
    for (int kk = 0; kk < 3; ++kk)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) Chr1[kk][a][b] = 0.5 * (dgt[a][kk][b] + dgt[b][kk][a] - dgt[kk][a][b]);
    for (int kk = 0; kk < 3; ++kk)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double s = 0.0;
                for (int l = 0; l < 3; ++l) s += gu[kk][l] * Chr1[l][a][b];
                Chr2[kk][a][b] = s;
            }
    for (int kk = 0; kk < 3; ++kk) {
        double s = 0.0;
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) s += gu[a][b] * Chr2[kk][a][b];
        Gtd[kk] = s;
    }
    /* Ricci scalar R = gu^ij W^2 R_ij (as in the right-hand side) */
    double Rt[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double t1 = 0.0, t2 = 0.0, t3 = 0.0, t4 = 0.0;
            for (int l = 0; l < 3; ++l)
                for (int m = 0; m < 3; ++m) t1 += gu[l][m] * ddgt[l][m][a][b];
            for (int c = 0; c < 3; ++c) t2 += gt[c][a] * dGt[b][c] + gt[c][b] * dGt[a][c];
            for (int c = 0; c < 3; ++c) t3 += Gtd[c] * (Chr1[a][b][c] + Chr1[b][a][c]);
            for (int l = 0; l < 3; ++l)
                for (int m = 0; m < 3; ++m)
                    for (int c = 0; c < 3; ++c)
                        t4 += gu[l][m] * (Chr2[c][l][a] * Chr1[b][c][m] + Chr2[c][l][b] * Chr1[a][c][m]
                                          + Chr2[c][a][m] * Chr1[c][l][b]);
            Rt[a][b] = -0.5 * t1 + 0.5 * t2 + 0.5 * t3 + t4;
        }
    (void)Gt;
    double DDW[3][3], trDDW = 0.0, dW2 = 0.0, R = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int c = 0; c < 3; ++c) s += Chr2[c][a][b] * dW[c];
            DDW[a][b] = ddW[a][b] - s;
        }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            trDDW += gu[a][b] * DDW[a][b];
            dW2 += gu[a][b] * dW[a] * dW[b];
        }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            R += gu[a][b] * (W * W * Rt[a][b] + W * (DDW[a][b] + gt[a][b] * trDDW) - 2.0 * gt[a][b] * dW2);
    /* raised At and At_ij At^ij */
    double Auu[3][3], AA = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double s = 0.0;
            for (int c = 0; c < 3; ++c)
                for (int d = 0; d < 3; ++d) s += gu[a][c] * gu[b][d] * At[c][d];
            Auu[a][b] = s;
        }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) AA += At[a][b] * Auu[a][b];
    out[0] = R - AA + 2.0 * K * K / 3.0;
    /* d_j gu^ia = -gu^ic gu^ad d_j gt_cd */
    double dgu[3][3][3]; /* [j][i][a] */
    for (int jj = 0; jj < 3; ++jj)
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double s = 0.0;
                for (int c = 0; c < 3; ++c)
                    for (int d = 0; d < 3; ++d) s += gu[a][c] * gu[b][d] * dgt[jj][c][d];
                dgu[jj][a][b] = -s;
            }
    for (int a = 0; a < 3; ++a) {
        double div = 0.0, chr = 0.0, aw = 0.0, gk = 0.0;
        for (int jj = 0; jj < 3; ++jj) {
            /* d_j At^aj */
            for (int c = 0; c < 3; ++c)
                for (int d = 0; d < 3; ++d)
                    div += gu[a][c] * gu[jj][d] * dAt[jj][c][d]
                         + At[c][d] * (dgu[jj][a][c] * gu[jj][d] + gu[a][c] * dgu[jj][jj][d]);
            for (int kk = 0; kk < 3; ++kk) chr += Chr2[a][jj][kk] * Auu[jj][kk] + Chr2[jj][jj][kk] * Auu[a][kk];
            aw += Auu[a][jj] * dW[jj];
            gk += gu[a][jj] * dK[jj];
        }
        out[1 + a] = W * W * (div + chr - 3.0 * aw / W - 2.0 * gk / 3.0);
    }
}

/* Constraints on every active point: c[m*sf + q] for m = H, M^x, M^y, M^z
   (ghost entries 0), and the volume-normalised L2 norms of paper Sec. 2.3,
   sqrt(sum C^2 dV / sum dV) over the active cells (cubic cells of one box:
   dV is constant), summed in plain (k, j, i) order. */
int oz_constraints(const double* u, double* c, double* norms, long sf, int nx, int ny, int nz, int ng, double dx,
                   double dy, double dz, double x0, double y0, double z0, int bc, const oz_params* p, int nthreads)
{
    grid g;
    if (!u || !c || !norms || !p || make_grid(&g, sf, nx, ny, nz, ng, dx, dy, dz, x0, y0, z0, bc)) return -1;
    for (long q = 0; q < 4 * sf; ++q) c[q] = 0.0;
#pragma omp parallel for schedule(static) num_threads(nthreads < 1 ? 1 : nthreads)
    for (int k = g.ng; k < g.ng + g.n[2]; ++k)
        for (int j = g.ng; j < g.ng + g.n[1]; ++j)
            for (int i = g.ng; i < g.ng + g.n[0]; ++i) {
                double out[4];
                constraints_point(u, &g, p, i, j, k, out);
                for (int m = 0; m < 4; ++m) c[m * sf + lin(&g, i, j, k)] = out[m];
            }
    for (int m = 0; m < 4; ++m) {
        double s = 0.0;
        for (int k = g.ng; k < g.ng + g.n[2]; ++k)
            for (int j = g.ng; j < g.ng + g.n[1]; ++j)
                for (int i = g.ng; i < g.ng + g.n[0]; ++i) {
                    double v = c[m * sf + lin(&g, i, j, k)];
                    s += v * v;
                }
        norms[m] = sqrt(s / ((double)g.n[0] * g.n[1] * g.n[2]));
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Sommerfeld right-hand side at an outer ghost point (Sec. 2.2.2):    */
/* d_t(rQ) + d_r(rQ) = 0 with Q = f - f_flat, speed 1                  */
/* ------------------------------------------------------------------ */
static double dsomm(const double* u, const grid* g, int f, const int P[3], int d)
{
    double c = fv(u, g, f, P, d, 0);
    if (P[d] - 1 >= 0 && P[d] + 1 < g->N[d])
        return (fv(u, g, f, P, d, 1) - fv(u, g, f, P, d, -1)) / (2.0 * g->h[d]);
    int s = (P[d] + 1 >= g->N[d]) ? 1 : -1; /* +1 at the upper edge: lean inward */
    double m1 = fv(u, g, f, P, d, -s), m2 = fv(u, g, f, P, d, -2 * s);
    return (double)s * (-4.0 * (m1 - c) + (m2 - c)) / (2.0 * g->h[d]);
}

static void somm_point(const double* u, const grid* g, int i, int j, int k, double out[NF])
{
    const int P[3] = {i, j, k};
    double x[3];
    for (int d = 0; d < 3; ++d) x[d] = g->x0[d] + (double)(P[d] - g->ng) * g->h[d];
    double r = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    for (int f = 0; f < NF; ++f) {
        double c = u[f * g->sf + lin(g, i, j, k)];
        double dr = 0.0;
        for (int d = 0; d < 3; ++d) dr += (x[d] / r) * dsomm(u, g, f, P, d);
        out[f] = -dr - (c - flat_value(f)) / r;
    }
}

static int is_active(const grid* g, int i, int j, int k)
{
    return i >= g->ng && i < g->ng + g->n[0] && j >= g->ng && j < g->ng + g->n[1] && k >= g->ng
        && k < g->ng + g->n[2];
}

/* points advanced in time: active points, plus the outer ghost points of
   Sommerfeld faces (all ghosts of a Sommerfeld box; those above the
   symmetry plane of an equatorial box) */
static int is_evolved(const grid* g, int i, int j, int k)
{
    if (is_active(g, i, j, k) || g->bc == BC_SOMMERFELD) return 1;
    return g->bc == BC_EQUATORIAL && k >= g->ng;
}

/* ------------------------------------------------------------------ */
/* Ghost fill (periodic wrap or copy from a fixed shell)              */
/* ------------------------------------------------------------------ */
static int wrap(int i, int ng, int n)
{
    int a = (i - ng) % n;
    if (a < 0) a += n;
    return a + ng;
}

static void ghosts(double* u, const double* shell, const grid* g)
{
    if (g->bc == BC_SOMMERFELD) return; /* ghosts are evolved, never filled */
    if (g->bc == BC_EQUATORIAL) {
        /* layers below the symmetry plane mirror those above it */
        for (int k = 0; k < g->ng; ++k)
            for (int j = 0; j < g->N[1]; ++j)
                for (int i = 0; i < g->N[0]; ++i)
                    for (int f = 0; f < NF; ++f)
                        u[f * g->sf + lin(g, i, j, k)] = z_parity(f) * u[f * g->sf + lin(g, i, j, 2 * g->ng - 1 - k)];
        return;
    }
    long nshell = (long)g->N[0] * g->N[1] * g->N[2] - (long)g->n[0] * g->n[1] * g->n[2];
    long q = 0; /* running index in the shell, points visited in (k, j, i) order */
    for (int k = 0; k < g->N[2]; ++k)
        for (int j = 0; j < g->N[1]; ++j)
            for (int i = 0; i < g->N[0]; ++i) {
                if (is_active(g, i, j, k)) continue;
                for (int f = 0; f < NF; ++f) {
                    double v;
                    if (g->bc == BC_PERIODIC)
                        v = u[f * g->sf + lin(g, wrap(i, g->ng, g->n[0]), wrap(j, g->ng, g->n[1]),
                                              wrap(k, g->ng, g->n[2]))];
                    else
                        v = shell[f * nshell + q];
                    u[f * g->sf + lin(g, i, j, k)] = v;
                }
                ++q;
            }
}

/* ------------------------------------------------------------------ */
/* Algebraic constraints det gt = 1, gt^ij At_ij = 0 at one point      */
/* ------------------------------------------------------------------ */
static void enforce_point(double* u, long sf, long q)
{
    double gt[3][3], At[3][3], gu[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            gt[a][b] = u[(IGT + sym[a][b]) * sf + q];
            At[a][b] = u[(IAT + sym[a][b]) * sf + q];
        }
    double scale = 1.0 / cbrt(det3(gt));
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) gt[a][b] *= scale;
    inv3(gt, gu);
    double tr = 0.0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) tr += gu[a][b] * At[a][b];
    for (int a = 0; a < 3; ++a)
        for (int b = a; b < 3; ++b) {
            u[(IGT + sym[a][b]) * sf + q] = gt[a][b];
            u[(IAT + sym[a][b]) * sf + q] = At[a][b] - gt[a][b] * tr / 3.0;
        }
}

/* ------------------------------------------------------------------ */
/* Exported entry points (C ABI, host pointers, called via ctypes)    */
/* ------------------------------------------------------------------ */
static int make_grid(grid* g, long sf, int nx, int ny, int nz, int ng, double dx, double dy, double dz,
                     double x0, double y0, double z0, int bc)
{
    if (nx < 1 || ny < 1 || nz < 1 || ng < 3 || !(dx > 0) || !(dy > 0) || !(dz > 0)) return -1;
    if (bc < 0 || bc > 3) return -1;
    g->n[0] = nx; g->n[1] = ny; g->n[2] = nz; g->ng = ng;
    for (int d = 0; d < 3; ++d) g->N[d] = g->n[d] + 2 * ng;
    if (sf < (long)g->N[0] * g->N[1] * g->N[2]) return -1;
    g->sf = sf;
    g->h[0] = dx; g->h[1] = dy; g->h[2] = dz;
    g->x0[0] = x0; g->x0[1] = y0; g->x0[2] = z0;
    g->bc = bc;
    return 0;
}

/* right-hand side on every evolved point; other ghost entries are 0 */
static void rhs_all(const double* u, double* rhs, const grid* g, const oz_params* p, int nthreads)
{
#pragma omp parallel for schedule(static) num_threads(nthreads)
    for (int k = 0; k < g->N[2]; ++k)
        for (int j = 0; j < g->N[1]; ++j)
            for (int i = 0; i < g->N[0]; ++i) {
                double out[NF];
                if (is_active(g, i, j, k))
                    rhs_point(u, g, p, i, j, k, out);
                else if (is_evolved(g, i, j, k))
                    somm_point(u, g, i, j, k, out);
                else
                    for (int f = 0; f < NF; ++f) out[f] = 0.0;
                for (int f = 0; f < NF; ++f) rhs[f * g->sf + lin(g, i, j, k)] = out[f];
            }
}

int oz_rhs(const double* u, double* rhs, long sf, int nx, int ny, int nz, int ng, double dx, double dy,
           double dz, double x0, double y0, double z0, int bc, const oz_params* p, int nthreads)
{
    grid g;
    if (!u || !rhs || !p || make_grid(&g, sf, nx, ny, nz, ng, dx, dy, dz, x0, y0, z0, bc)) return -1;
    rhs_all(u, rhs, &g, p, nthreads < 1 ? 1 : nthreads);
    return 0;
}

/* right-hand side at a list of stored-index points pts[3*q] = (i, j, k);
   out[q*NF + f] */
int oz_rhs_points(const double* u, long sf, int nx, int ny, int nz, int ng, double dx, double dy, double dz,
                  double x0, double y0, double z0, int bc, const oz_params* p, const int* pts, long npts,
                  double* out, int nthreads)
{
    grid g;
    if (!u || !p || !pts || !out || make_grid(&g, sf, nx, ny, nz, ng, dx, dy, dz, x0, y0, z0, bc)) return -1;
    for (long q = 0; q < npts; ++q)
        for (int d = 0; d < 3; ++d)
            if (pts[3 * q + d] < 0 || pts[3 * q + d] >= g.N[d]) return -1;
#pragma omp parallel for schedule(static) num_threads(nthreads < 1 ? 1 : nthreads)
    for (long q = 0; q < npts; ++q) {
        int i = pts[3 * q], j = pts[3 * q + 1], k = pts[3 * q + 2];
        if (is_active(&g, i, j, k))
            rhs_point(u, &g, p, i, j, k, out + q * NF);
        else if (is_evolved(&g, i, j, k))
            somm_point(u, &g, i, j, k, out + q * NF);
        else
            for (int f = 0; f < NF; ++f) out[q * NF + f] = 0.0;
    }
    return 0;
}

int oz_apply_ghosts(double* u, const double* shell, long sf, int nx, int ny, int nz, int ng, int bc)
{
    grid g;
    if (!u || make_grid(&g, sf, nx, ny, nz, ng, 1.0, 1.0, 1.0, 0.0, 0.0, 0.0, bc)) return -1;
    if (bc == BC_COPY && !shell) return -1;
    ghosts(u, shell, &g);
    return 0;
}

/* enforce the algebraic constraints on the evolved points of u (active
   points, plus the Sommerfeld-face ghosts) */
int oz_enforce(double* u, long sf, int nx, int ny, int nz, int ng, int bc)
{
    grid g;
    if (!u || make_grid(&g, sf, nx, ny, nz, ng, 1.0, 1.0, 1.0, 0.0, 0.0, 0.0, bc)) return -1;
    for (int k = 0; k < g.N[2]; ++k)
        for (int j = 0; j < g.N[1]; ++j)
            for (int i = 0; i < g.N[0]; ++i)
                if (is_evolved(&g, i, j, k)) enforce_point(u, sf, lin(&g, i, j, k));
    return 0;
}

/* One explicit stage at sampled points: out = enforce(u_n + c*dt*rhs(u_in)).
   u_in must have valid ghosts.  out[q*NF + f]. */
int oz_stage_points(const double* u_in, const double* u_n, double c_dt, long sf, int nx, int ny, int nz, int ng,
                    double dx, double dy, double dz, double x0, double y0, double z0, int bc, const oz_params* p,
                    const int* pts, long npts, double* out, int nthreads)
{
    int rc = oz_rhs_points(u_in, sf, nx, ny, nz, ng, dx, dy, dz, x0, y0, z0, bc, p, pts, npts, out, nthreads);
    if (rc) return rc;
    for (long q = 0; q < npts; ++q) {
        long s = ((long)pts[3 * q + 2] * (ny + 2 * ng) + pts[3 * q + 1]) * (nx + 2 * ng) + pts[3 * q];
        double tmp[NF];
        for (int f = 0; f < NF; ++f) tmp[f] = u_n[f * sf + s] + c_dt * out[q * NF + f];
        enforce_point(tmp, 1, 0);
        for (int f = 0; f < NF; ++f) out[q * NF + f] = tmp[f];
    }
    return 0;
}

/* Classical RK4 (Sec. 2.2), nsteps steps of size dt, in place on u.
   k1 = F(u); u1 = u + dt/2 k1; k2 = F(u1); u2 = u + dt/2 k2; k3 = F(u2);
   u3 = u + dt k3; k4 = F(u3); u <- u + dt/6 (((k1 + 2 k2) + 2 k3) + k4).
   Every stage state is enforced on its evolved points and its ghosts filled. */
int oz_rk4(double* u, const double* shell, long sf, int nx, int ny, int nz, int ng, double dx, double dy, double dz,
           double x0, double y0, double z0, int bc, const oz_params* p, double dt, int nsteps, int nthreads)
{
    grid g;
    if (!u || !p || make_grid(&g, sf, nx, ny, nz, ng, dx, dy, dz, x0, y0, z0, bc)) return -1;
    if (bc == BC_COPY && !shell) return -1;
    if (!(dt > 0) || nsteps < 0) return -1;
    int nt = nthreads < 1 ? 1 : nthreads;
    size_t bytes = (size_t)NF * (size_t)sf * sizeof(double);
    double* us = malloc(bytes);
    double* kk[4];
    for (int s = 0; s < 4; ++s) kk[s] = malloc(bytes);
    if (!us || !kk[0] || !kk[1] || !kk[2] || !kk[3]) {
        free(us);
        for (int s = 0; s < 4; ++s) free(kk[s]);
        return -3;
    }
    const double cstage[3] = {0.5, 0.5, 1.0};
    for (int step = 0; step < nsteps; ++step) {
        ghosts(u, shell, &g);
        for (int s = 0; s < 4; ++s) {
            const double* src = (s == 0) ? u : us;
            rhs_all(src, kk[s], &g, p, nt);
            if (s == 3) break;
#pragma omp parallel for schedule(static) num_threads(nt)
            for (int k = 0; k < g.N[2]; ++k)
                for (int j = 0; j < g.N[1]; ++j)
                    for (int i = 0; i < g.N[0]; ++i) {
                        long q = lin(&g, i, j, k);
                        int evolved = is_evolved(&g, i, j, k);
                        for (int f = 0; f < NF; ++f)
                            us[f * sf + q] = evolved ? u[f * sf + q] + cstage[s] * dt * kk[s][f * sf + q]
                                                     : u[f * sf + q];
                        if (evolved) enforce_point(us, sf, q);
                    }
            ghosts(us, shell, &g);
        }
#pragma omp parallel for schedule(static) num_threads(nt)
        for (int k = 0; k < g.N[2]; ++k)
            for (int j = 0; j < g.N[1]; ++j)
                for (int i = 0; i < g.N[0]; ++i) {
                    long q = lin(&g, i, j, k);
                    if (!is_evolved(&g, i, j, k)) continue;
                    for (int f = 0; f < NF; ++f) {
                        long o = f * sf + q;
                        u[o] = u[o] + dt / 6.0 * (((kk[0][o] + 2.0 * kk[1][o]) + 2.0 * kk[2][o]) + kk[3][o]);
                    }
                    enforce_point(u, sf, q);
                }
        ghosts(u, shell, &g);
    }
    free(us);
    for (int s = 0; s < 4; ++s) free(kk[s]);
    return 0;
}

/* 1-D stencil probe for the stencil pins: applies one operator at every
   interior point q in [3, n-3) of f[0..n).  op: 0 = D1, 1 = D2, 2 = upwind
   with shift sign of beta_sign, 3 = KO6 (undivided). */
int oz_stencil_1d(int op, const double* f, int n, double h, double beta_sign, double* out)
{
    if (!f || !out || n < 7 || !(h > 0) || op < 0 || op > 3) return -1;
    /* copy f into a grid that is n long in x and 7 deep in y and z */
    double* buf = calloc((size_t)n * 49, sizeof(double));
    if (!buf) return -3;
    grid h1;
    make_grid(&h1, (long)n * 49, n - 6, 1, 1, 3, h, 1.0, 1.0, 0.0, 0.0, 0.0, BC_COPY);
    for (int k = 0; k < 7; ++k)
        for (int j = 0; j < 7; ++j)
            for (int i = 0; i < n; ++i) buf[lin(&h1, i, j, k)] = f[i];
    for (int i = 0; i < n; ++i) out[i] = 0.0;
    for (int i = 3; i < n - 3; ++i) {
        int P[3] = {i, 3, 3};
        switch (op) {
        case 0: out[i] = D1(buf, &h1, 0, P, 0); break;
        case 1: out[i] = D2(buf, &h1, 0, P, 0); break;
        case 2: out[i] = DUP(buf, &h1, 0, P, 0, beta_sign); break;
        default: out[i] = KO6(buf, &h1, 0, P, 0); break;
        }
    }
    free(buf);
    return 0;
}

/* 2-D probe of the mixed derivative D1_x(D1_y f) on an nx-by-ny array
   (x fastest), at interior points [3, n-3) in both directions */
int oz_mixed_2d(const double* f, int nx, int ny, double hx, double hy, double* out)
{
    if (!f || !out || nx < 7 || ny < 7 || !(hx > 0) || !(hy > 0)) return -1;
    grid g;
    make_grid(&g, (long)nx * ny * 7, nx - 6, ny - 6, 1, 3, hx, hy, 1.0, 0.0, 0.0, 0.0, BC_COPY);
    double* buf = calloc((size_t)nx * ny * 7, sizeof(double));
    if (!buf) return -3;
    for (int k = 0; k < 7; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) buf[lin(&g, i, j, k)] = f[j * nx + i];
    for (int q = 0; q < nx * ny; ++q) out[q] = 0.0;
    for (int j = 3; j < ny - 3; ++j)
        for (int i = 3; i < nx - 3; ++i) {
            int P[3] = {i, j, 3};
            out[j * nx + i] = DMIX(buf, &g, 0, P, 0, 1);
        }
    free(buf);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Box-in-box hierarchy with Berger-Oliger time subcycling (Sec.       */
/* 2.2.1).  The hierarchy is a list of patches; patch 0 is the root    */
/* (coarsest level, with its own boundary), every other patch names    */
/* its parent, which refines it 2:1 on a cell-centred grid (child      */
/* centres sit h_parent/4 from parent centres).  All patches at one    */
/* depth share the depth's lattice and step together: two steps of     */
/* half the size per parent step.  Fixed levels are single patches;    */
/* moving levels hold one patch per tracked object.                    */
/*                                                                     */
/* Transfers between depths: a child's ghost zone is filled by 6th-     */
/* order Lagrange interpolation in space of its parent, interpolated   */
/* in time between the parent's time levels (2nd order, 1st order      */
/* while the parent has no earlier level); after the children have     */
/* caught up, every coarse cell covered by a child's active region is  */
/* overwritten by a 4th-order Lagrange interpolation of the child data */
/* (the average over the children covering it, where several do).     */
/*                                                                     */
/* Exchange between patches at one depth: where two active regions     */
/* overlap, each takes the average of all of them; a ghost point that  */
/* lies in another patch's active region takes that patch's value (the */
/* first such patch in index order); ghost over ghost changes nothing. */
/*                                                                     */
/* Readings (also in the design notes): the child's lower faces        */
/* coincide with parent cell faces (F = parent active cell index of    */
/* the face); the restriction stencil reaches one child ghost layer,   */
/* which is filled by prolongation and exchange at the new time first; */
/* stage inputs get their ghosts (prolongation, then exchange) at the  */
/* stage time; overlapping active cells are averaged once per step,    */
/* after the last stage.                                               */
/* ------------------------------------------------------------------ */

#define OZ_MAXPATCH 32

typedef struct {
    double* u;    /* state, advanced in place */
    double* prev; /* this patch one step earlier (kept for the time interpolation of its children) */
    long sf;
    int n[3];
    int ng;
    double h[3];
    double x0[3];
    int F[3];     /* patches >= 1: lower face in the parent's active cell index */
    int bc;       /* root: its own boundary kind; other patches: ignored (filled from the parent) */
    int has_prev; /* in/out: prev holds a valid earlier time level */
    int parent;   /* index of the parent patch, below the patch's own; -1 for the root (patch 0) */
    int obj;      /* moving patches: the tracked object they follow; -1 for a fixed patch */
} oz_level;

/* the hierarchy during an advance: geometry derived from the patches and
   the per-patch work arrays */
typedef struct {
    oz_level* lv;
    int np;
    int depth[OZ_MAXPATCH];
    int off[OZ_MAXPATCH][3]; /* lattice index of the first active cell at the patch's depth */
    int plane[OZ_MAXPATCH];  /* the patch's lower z face is the symmetry plane of an equatorial root */
    int maxdepth;
    grid g[OZ_MAXPATCH];
    double* cur[OZ_MAXPATCH]; /* the patch at the start of its current step */
    double* us[OZ_MAXPATCH];  /* stage input */
    double* kk[OZ_MAXPATCH][4];
    const oz_params* p;
    double dt0;
    int nt;
    int nobj;
    double* xp;              /* 3 per object, in/out */
    int tp[OZ_MAXPATCH];     /* per object: the patch it is tracked on */
    double b0[OZ_MAXPATCH][3], xs[OZ_MAXPATCH][3];
} hierarchy;

/* Lagrange weights of the m nodes at the point x */
static void lagrange_weights(const double* nodes, int m, double x, double* w)
{
    for (int a = 0; a < m; ++a) {
        double num = 1.0, den = 1.0;
        for (int b = 0; b < m; ++b)
            if (b != a) {
                num *= x - nodes[b];
                den *= nodes[a] - nodes[b];
            }
        w[a] = num / den;
    }
}

/* child active index a along one direction -> first parent active index
   of the 6-point stencil and its weights.  Child cell a lies in parent cell
   F + floor(a/2), a quarter parent cell below (a even) or above (a odd)
   its centre; the stencil takes three parent cells on the near side and
   two on the far side plus the containing one. */
static int prolong_1d(int a, int F, double w[6])
{
    int half = a >= 0 ? a / 2 : -((1 - a) / 2); /* floor(a / 2) */
    int odd = a - 2 * half;
    double nodes[6];
    int first = odd ? -2 : -3;
    for (int m = 0; m < 6; ++m) nodes[m] = (double)(first + m);
    lagrange_weights(nodes, 6, odd ? 0.25 : -0.25, w);
    return F + half + first;
}

static void make_level_grid(grid* g, const oz_level* L, int bc)
{
    make_grid(g, L->sf, L->n[0], L->n[1], L->n[2], L->ng, L->h[0], L->h[1], L->h[2], L->x0[0], L->x0[1],
              L->x0[2], bc);
}

/* Fill every ghost point of the child from the parent time levels
   pa[0..3) combined with the time weights wt (a NULL level has weight 0). */
static void prolong_ghosts(const grid* gp, const double* const pa[3], const double wt[3], const grid* gc,
                           double* uc, const int F[3], int refl, int nt)
{
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int k = 0; k < gc->N[2]; ++k)
        for (int j = 0; j < gc->N[1]; ++j)
            for (int i = 0; i < gc->N[0]; ++i) {
                if (is_active(gc, i, j, k)) continue;
                double wx[6], wy[6], wz[6];
                int lx = prolong_1d(i - gc->ng, F[0], wx) + gp->ng;
                int ly = prolong_1d(j - gc->ng, F[1], wy) + gp->ng;
                int lz = prolong_1d(k - gc->ng, F[2], wz) + gp->ng;
                for (int f = 0; f < NF; ++f) {
                    double s = 0.0;
                    for (int c = 0; c < 6; ++c) {
                        /* refl: parent layers below the symmetry plane are the
                           mirror images of those above it */
                        int kz = lz + c, neg = 0;
                        if (refl && kz < gp->ng) {
                            kz = 2 * gp->ng - 1 - kz;
                            neg = z_parity(f) < 0;
                        }
                        for (int b = 0; b < 6; ++b)
                            for (int a = 0; a < 6; ++a) {
                                long q = f * gp->sf + lin(gp, lx + a, ly + b, kz);
                                double v = 0.0;
                                for (int t = 0; t < 3; ++t)
                                    if (pa[t]) v += wt[t] * pa[t][q];
                                s += wz[c] * wy[b] * wx[a] * (neg ? -v : v);
                            }
                    }
                    uc[f * gc->sf + lin(gc, i, j, k)] = s;
                }
            }
}

/* 4th-order Lagrange interpolation of field f of the child to the centre
   of a parent cell: child cells (ci..ci+3) x (cj..) x (ck..) (stored
   indices), nodes at -3/2, -1/2, 1/2, 3/2 child cells from that centre */
static double restrict_value(const grid* gc, const double* uc, int f, int ci, int cj, int ck)
{
    static const double nodes[4] = {-1.5, -0.5, 0.5, 1.5};
    double r[4];
    lagrange_weights(nodes, 4, 0.0, r);
    double s = 0.0;
    for (int z = 0; z < 4; ++z)
        for (int y = 0; y < 4; ++y)
            for (int x = 0; x < 4; ++x) s += r[z] * r[y] * r[x] * uc[f * gc->sf + lin(gc, ci + x, cj + y, ck + z)];
    return s;
}

/* Overwrite every parent active cell covered by the child's active region
   with the restriction of the child (probe of a single parent/child pair) */
static void restrict_to_parent(const grid* gc, const double* uc, const grid* gp, double* up, const int F[3], int nt)
{
    const int m0 = gc->n[0] / 2, m1 = gc->n[1] / 2, m2 = gc->n[2] / 2;
#pragma omp parallel for schedule(static) num_threads(nt)
    for (int c = 0; c < m2; ++c)
        for (int b = 0; b < m1; ++b)
            for (int a = 0; a < m0; ++a) {
                /* child active cells 2a-1 .. 2a+2 (and likewise in y, z) */
                int ci = 2 * a - 1 + gc->ng, cj = 2 * b - 1 + gc->ng, ck = 2 * c - 1 + gc->ng;
                long qp = lin(gp, F[0] + a + gp->ng, F[1] + b + gp->ng, F[2] + c + gp->ng);
                for (int f = 0; f < NF; ++f) up[f * gp->sf + qp] = restrict_value(gc, uc, f, ci, cj, ck);
            }
}

/* weights of the parent levels (earlier, start, end of the parent step)
   at the fraction theta of the parent step */
static void time_weights(double theta, int quadratic, double wt[3])
{
    if (quadratic) {
        static const double nodes[3] = {-1.0, 0.0, 1.0};
        lagrange_weights(nodes, 3, theta, wt);
    } else {
        static const double nodes[2] = {0.0, 1.0};
        wt[0] = 0.0;
        lagrange_weights(nodes, 2, theta, wt + 1);
    }
}

/* ---- hierarchy geometry ---- */

/* depths, lattice offsets and grids of every patch; -1 if the patch list
   is not a valid hierarchy */
static int hier_geometry(hierarchy* H)
{
    H->maxdepth = 0;
    for (int q = 0; q < H->np; ++q) {
        const oz_level* L = &H->lv[q];
        if (!L->u || !L->prev) return -1;
        if (q == 0) {
            if (L->parent != -1 || L->bc == BC_COPY) return -1; /* the root needs a boundary of its own */
            H->depth[0] = 0;
            H->plane[0] = L->bc == BC_EQUATORIAL;
            for (int d = 0; d < 3; ++d) H->off[0][d] = 0;
            if (make_grid(&H->g[0], L->sf, L->n[0], L->n[1], L->n[2], L->ng, L->h[0], L->h[1], L->h[2], L->x0[0],
                          L->x0[1], L->x0[2], L->bc))
                return -1;
            continue;
        }
        if (L->parent < 0 || L->parent >= q) return -1;
        const oz_level* P = &H->lv[L->parent];
        H->depth[q] = H->depth[L->parent] + 1;
        if (H->depth[q] > H->maxdepth) H->maxdepth = H->depth[q];
        H->plane[q] = H->plane[L->parent] && L->F[2] == 0;
        if (make_grid(&H->g[q], L->sf, L->n[0], L->n[1], L->n[2], L->ng, L->h[0], L->h[1], L->h[2], L->x0[0],
                      L->x0[1], L->x0[2], BC_COPY))
            return -1;
        for (int d = 0; d < 3; ++d) {
            if (L->n[d] % 2 || L->h[d] != 0.5 * P->h[d]) return -1;
            /* prolongation stencil of every child ghost inside the parent's active cells */
            double w[6];
            int lo = prolong_1d(-L->ng, L->F[d], w), hi = prolong_1d(L->n[d] + L->ng - 1, L->F[d], w) + 5;
            if (d == 2 && H->plane[q]) lo = lo < 0 ? -1 - lo : lo; /* reflected across the plane */
            if (lo < 0 || lo >= P->n[d] || hi >= P->n[d]) return -1;
            /* child active cell a sits at lattice index 2 (parent's first cell + F) + a */
            H->off[q][d] = 2 * (H->off[L->parent][d] + L->F[d]);
        }
    }
    return 0;
}

static int in_active(const hierarchy* H, int q, const int G[3])
{
    for (int d = 0; d < 3; ++d) {
        int a = G[d] - H->off[q][d];
        if (a < 0 || a >= H->lv[q].n[d]) return 0;
    }
    return 1;
}

/* stored index of the lattice point G in patch q */
static long lattice_lin(const hierarchy* H, int q, const int G[3])
{
    const int ng = H->lv[q].ng;
    return lin(&H->g[q], G[0] - H->off[q][0] + ng, G[1] - H->off[q][1] + ng, G[2] - H->off[q][2] + ng);
}

/* Exchange at depth d, averaging: every lattice cell in the active regions
   of several patches gets their mean in all of them.  The first patch (in
   index order) that holds the cell does the work, so each cell is handled
   once. */
static void exchange_average(hierarchy* H, int d, double* const* arr)
{
    for (int a = 0; a < H->np; ++a) {
        if (H->depth[a] != d) continue;
        const oz_level* A = &H->lv[a];
#pragma omp parallel for schedule(static) num_threads(H->nt)
        for (int k = 0; k < A->n[2]; ++k)
            for (int j = 0; j < A->n[1]; ++j)
                for (int i = 0; i < A->n[0]; ++i) {
                    const int G[3] = {H->off[a][0] + i, H->off[a][1] + j, H->off[a][2] + k};
                    int first = -1, cnt = 0;
                    for (int b = 0; b < H->np; ++b)
                        if (H->depth[b] == d && in_active(H, b, G)) {
                            if (first < 0) first = b;
                            ++cnt;
                        }
                    if (first != a || cnt < 2) continue;
                    for (int f = 0; f < NF; ++f) {
                        double s = 0.0;
                        for (int b = 0; b < H->np; ++b)
                            if (H->depth[b] == d && in_active(H, b, G)) s += arr[b][f * H->lv[b].sf + lattice_lin(H, b, G)];
                        const double v = s / cnt;
                        for (int b = 0; b < H->np; ++b)
                            if (H->depth[b] == d && in_active(H, b, G)) arr[b][f * H->lv[b].sf + lattice_lin(H, b, G)] = v;
                    }
                }
    }
}

/* Exchange at depth d, ghosts: a ghost point of a patch that lies in the
   active region of another patch of the depth takes its value (the first
   such patch in index order). */
static void exchange_ghosts(hierarchy* H, int d, double* const* arr)
{
    for (int b = 0; b < H->np; ++b) {
        if (H->depth[b] != d) continue;
        const grid* g = &H->g[b];
#pragma omp parallel for schedule(static) num_threads(H->nt)
        for (int k = 0; k < g->N[2]; ++k)
            for (int j = 0; j < g->N[1]; ++j)
                for (int i = 0; i < g->N[0]; ++i) {
                    if (is_active(g, i, j, k)) continue;
                    const int G[3] = {H->off[b][0] + i - g->ng, H->off[b][1] + j - g->ng, H->off[b][2] + k - g->ng};
                    for (int a = 0; a < H->np; ++a) {
                        if (a == b || H->depth[a] != d || !in_active(H, a, G)) continue;
                        const long qa = lattice_lin(H, a, G), qb = lin(g, i, j, k);
                        for (int f = 0; f < NF; ++f) arr[b][f * g->sf + qb] = arr[a][f * H->lv[a].sf + qa];
                        break;
                    }
                }
    }
}

/* ghosts of arr[q] for every patch q at depth d at the fraction theta of
   the parent step (the root: its own boundary), then the exchange */
static void fill_depth(hierarchy* H, int d, double* const* arr, double theta)
{
    for (int q = 0; q < H->np; ++q) {
        if (H->depth[q] != d) continue;
        if (q == 0) {
            ghosts(arr[q], NULL, &H->g[q]);
            continue;
        }
        const int P = H->lv[q].parent;
        const oz_level* LP = &H->lv[P];
        double wt[3];
        time_weights(theta, LP->has_prev, wt);
        const double* pa[3] = {LP->has_prev ? LP->prev : NULL, H->cur[P], LP->u};
        prolong_ghosts(&H->g[P], pa, wt, &H->g[q], arr[q], H->lv[q].F, H->plane[q], H->nt);
    }
    exchange_ghosts(H, d, arr);
    /* layers below the symmetry plane: mirror images of the patch's own */
    for (int q = 1; q < H->np; ++q)
        if (H->depth[q] == d && H->plane[q]) {
            grid ge = H->g[q];
            ge.bc = BC_EQUATORIAL;
            ghosts(arr[q], NULL, &ge);
        }
}

/* Every active cell of a patch at depth d covered by the active region of
   a patch at depth d+1 takes the restriction of that child (the mean over
   the children that cover it). */
static void restrict_depth(hierarchy* H, int d)
{
    for (int q = 0; q < H->np; ++q) {
        if (H->depth[q] != d) continue;
        const oz_level* P = &H->lv[q];
#pragma omp parallel for schedule(static) num_threads(H->nt)
        for (int k = 0; k < P->n[2]; ++k)
            for (int j = 0; j < P->n[1]; ++j)
                for (int i = 0; i < P->n[0]; ++i) {
                    const int G[3] = {H->off[q][0] + i, H->off[q][1] + j, H->off[q][2] + k};
                    double s[NF];
                    int cnt = 0;
                    for (int c = 0; c < H->np; ++c) {
                        if (H->depth[c] != d + 1) continue;
                        int ac[3], cov = 1;
                        for (int e = 0; e < 3; ++e) {
                            /* the parent cell spans child cells ac, ac+1 */
                            ac[e] = 2 * G[e] - H->off[c][e];
                            cov &= ac[e] >= 0 && ac[e] + 1 < H->lv[c].n[e];
                        }
                        if (!cov) continue;
                        const grid* gc = &H->g[c];
                        for (int f = 0; f < NF; ++f) {
                            double v = restrict_value(gc, H->lv[c].u, f, ac[0] - 1 + gc->ng, ac[1] - 1 + gc->ng,
                                                      ac[2] - 1 + gc->ng);
                            s[f] = cnt ? s[f] + v : v;
                        }
                        ++cnt;
                    }
                    if (!cnt) continue;
                    const long qp = lin(&H->g[q], i + P->ng, j + P->ng, k + P->ng);
                    for (int f = 0; f < NF; ++f) P->u[f * P->sf + qp] = cnt == 1 ? s[f] : s[f] / cnt;
                }
    }
}

static int interp_beta(const oz_level* L, const double x[3], int refl, double b[3]);

/* one RK4 step of every patch at depth d (the textbook form of oz_rk4),
   ghosts of every stage input filled at that stage's time, then the two
   steps of depth d+1 and the restriction */
static int bo_depth(hierarchy* H, int d, double theta0)
{
    const double dt = H->dt0 / (double)(1L << d);
    /* stage times in units of the parent step: theta0 + {0, 1/4, 1/4, 1/2} */
    const double cstage[3] = {0.5, 0.5, 1.0};
    double* uarr[OZ_MAXPATCH];
    for (int q = 0; q < H->np; ++q) uarr[q] = H->lv[q].u;
    fill_depth(H, d, uarr, theta0);
    for (int q = 0; q < H->np; ++q)
        if (H->depth[q] == d) memcpy(H->cur[q], H->lv[q].u, (size_t)NF * (size_t)H->lv[q].sf * sizeof(double));
    /* puncture tracking on each object's finest patch: Heun's method for
       dx/dt = -beta, beta at the start of the step at x, at its end at the
       predicted point */
    for (int o = 0; o < H->nobj; ++o) {
        if (H->depth[H->tp[o]] != d) continue;
        if (interp_beta(&H->lv[H->tp[o]], H->xp + 3 * o, H->plane[H->tp[o]], H->b0[o])) return -2;
        for (int e = 0; e < 3; ++e) H->xs[o][e] = H->xp[3 * o + e] - dt * H->b0[o][e];
    }
    for (int s = 0; s < 4; ++s) {
        for (int q = 0; q < H->np; ++q)
            if (H->depth[q] == d) rhs_all(s == 0 ? H->lv[q].u : H->us[q], H->kk[q][s], &H->g[q], H->p, H->nt);
        if (s == 3) break;
        for (int q = 0; q < H->np; ++q) {
            if (H->depth[q] != d) continue;
            const grid* g = &H->g[q];
            const double* u = H->lv[q].u;
            double* us = H->us[q];
            const double* kq = H->kk[q][s];
            const long sf = g->sf;
#pragma omp parallel for schedule(static) num_threads(H->nt)
            for (int k = 0; k < g->N[2]; ++k)
                for (int j = 0; j < g->N[1]; ++j)
                    for (int i = 0; i < g->N[0]; ++i) {
                        long x = lin(g, i, j, k);
                        int ev = is_evolved(g, i, j, k);
                        for (int f = 0; f < NF; ++f)
                            us[f * sf + x] = ev ? u[f * sf + x] + cstage[s] * dt * kq[f * sf + x] : u[f * sf + x];
                        if (ev) enforce_point(us, sf, x);
                    }
        }
        fill_depth(H, d, H->us, theta0 + 0.5 * cstage[s]);
    }
    for (int q = 0; q < H->np; ++q) {
        if (H->depth[q] != d) continue;
        const grid* g = &H->g[q];
        double* u = H->lv[q].u;
        double* const* kk = H->kk[q];
        const long sf = g->sf;
#pragma omp parallel for schedule(static) num_threads(H->nt)
        for (int k = 0; k < g->N[2]; ++k)
            for (int j = 0; j < g->N[1]; ++j)
                for (int i = 0; i < g->N[0]; ++i) {
                    long x = lin(g, i, j, k);
                    if (!is_evolved(g, i, j, k)) continue;
                    for (int f = 0; f < NF; ++f) {
                        long o = f * sf + x;
                        u[o] = u[o] + dt / 6.0 * (((kk[0][o] + 2.0 * kk[1][o]) + 2.0 * kk[2][o]) + kk[3][o]);
                    }
                    enforce_point(u, sf, x);
                }
    }
    exchange_average(H, d, uarr);
    fill_depth(H, d, uarr, theta0 + 0.5);
    for (int o = 0; o < H->nobj; ++o) {
        if (H->depth[H->tp[o]] != d) continue;
        double b1[3];
        if (interp_beta(&H->lv[H->tp[o]], H->xs[o], H->plane[H->tp[o]], b1)) return -2;
        for (int e = 0; e < 3; ++e) H->xp[3 * o + e] -= 0.5 * dt * (H->b0[o][e] + b1[e]);
    }
    if (d < H->maxdepth) {
        int rc;
        if ((rc = bo_depth(H, d + 1, 0.0)) || (rc = bo_depth(H, d + 1, 0.5))) return rc;
        fill_depth(H, d + 1, uarr, 1.0);
        restrict_depth(H, d);
        fill_depth(H, d, uarr, theta0 + 0.5);
    }
    for (int q = 0; q < H->np; ++q) {
        if (H->depth[q] != d) continue;
        memcpy(H->lv[q].prev, H->cur[q], (size_t)NF * (size_t)H->lv[q].sf * sizeof(double));
        H->lv[q].has_prev = 1;
    }
    return 0;
}

static void hier_release(hierarchy* H)
{
    for (int q = 0; q < OZ_MAXPATCH; ++q) {
        free(H->cur[q]);
        free(H->us[q]);
        for (int s = 0; s < 4; ++s) free(H->kk[q][s]);
    }
}

/* validate the patches and allocate the work arrays; objects 0..nobj-1
   are tracked on their deepest patch (exactly one patch of each object at
   its deepest depth) */
static int hier_init(hierarchy* H, oz_level* lv, int np, const oz_params* p, double dt0, int nobj, double* xp,
                     int nthreads)
{
    memset(H, 0, sizeof(*H));
    if (!lv || np < 1 || np > OZ_MAXPATCH || nobj < 0 || nobj > OZ_MAXPATCH || (nobj && !xp)) return -1;
    H->lv = lv;
    H->np = np;
    H->p = p;
    H->dt0 = dt0;
    H->nt = nthreads < 1 ? 1 : nthreads;
    H->nobj = nobj;
    H->xp = xp;
    if (hier_geometry(H)) return -1;
    for (int o = 0; o < nobj; ++o) {
        H->tp[o] = -1;
        int dmax = -1, count = 0;
        for (int q = 0; q < np; ++q) {
            if (lv[q].obj != o) continue;
            if (H->depth[q] > dmax) {
                dmax = H->depth[q];
                H->tp[o] = q;
                count = 1;
            } else if (H->depth[q] == dmax) {
                ++count;
            }
        }
        if (H->tp[o] < 0 || count != 1) return -1;
    }
    for (int q = 0; q < np; ++q)
        if (lv[q].obj >= nobj && nobj > 0) return -1;
    for (int q = 0; q < np; ++q) {
        const size_t bytes = (size_t)NF * (size_t)lv[q].sf * sizeof(double);
        H->cur[q] = malloc(bytes);
        H->us[q] = malloc(bytes);
        int ok = H->cur[q] && H->us[q];
        for (int s = 0; s < 4; ++s) ok &= (H->kk[q][s] = malloc(bytes)) != NULL;
        if (!ok) {
            hier_release(H);
            return -3;
        }
    }
    return 0;
}

/* Advance the hierarchy lv[0..np) by nsteps steps of the root (size dt0;
   a patch at depth d takes 2^d steps of dt0 / 2^d per root step). */
int oz_bo_advance(oz_level* lv, int np, const oz_params* p, double dt0, int nsteps, int nthreads)
{
    hierarchy H;
    if (!p || !(dt0 > 0) || nsteps < 0) return -1;
    int rc = hier_init(&H, lv, np, p, dt0, 0, NULL, nthreads);
    if (rc) return rc;
    for (int s = 0; s < nsteps && !rc; ++s) rc = bo_depth(&H, 0, 0.0);
    hier_release(&H);
    return rc;
}

/* Probes for the pins: prolongation of the parent (three time levels,
   pa[t] may be NULL) into every ghost of the child, and restriction. */
int oz_prolong(const double* pa0, const double* pa1, const double* pa2, const double* wt, long sfp, const int* np,
               int ngp, double* uc, long sfc, const int* nc, int ngc, const int* F, int refl, int nthreads)
{
    grid gp, gc;
    if (!uc || !wt || !np || !nc || !F) return -1;
    if (make_grid(&gp, sfp, np[0], np[1], np[2], ngp, 1.0, 1.0, 1.0, 0.0, 0.0, 0.0, BC_COPY)) return -1;
    if (make_grid(&gc, sfc, nc[0], nc[1], nc[2], ngc, 0.5, 0.5, 0.5, 0.0, 0.0, 0.0, BC_COPY)) return -1;
    for (int d = 0; d < 3; ++d) {
        double w[6];
        int lo = prolong_1d(-ngc, F[d], w) + ngp, hi = prolong_1d(nc[d] + ngc - 1, F[d], w) + 5 + ngp;
        if (d == 2 && refl) lo = lo < ngp ? 2 * ngp - 1 - lo : lo; /* reflected across the plane */
        if (lo < 0 || lo >= gp.N[d] || hi >= gp.N[d]) return -1;
    }
    const double* pa[3] = {pa0, pa1, pa2};
    prolong_ghosts(&gp, pa, wt, &gc, uc, F, refl != 0, nthreads < 1 ? 1 : nthreads);
    return 0;
}

int oz_restrict(const double* uc, long sfc, const int* nc, int ngc, double* up, long sfp, const int* np, int ngp,
                const int* F, int nthreads)
{
    grid gp, gc;
    if (!uc || !up || !np || !nc || !F) return -1;
    if (make_grid(&gp, sfp, np[0], np[1], np[2], ngp, 1.0, 1.0, 1.0, 0.0, 0.0, 0.0, BC_COPY)) return -1;
    if (make_grid(&gc, sfc, nc[0], nc[1], nc[2], ngc, 0.5, 0.5, 0.5, 0.0, 0.0, 0.0, BC_COPY)) return -1;
    for (int d = 0; d < 3; ++d)
        if (nc[d] % 2 || F[d] < 0 || F[d] + nc[d] / 2 > np[d]) return -1;
    restrict_to_parent(&gc, uc, &gp, up, F, nthreads < 1 ? 1 : nthreads);
    return 0;
}

/* the weights themselves, for the pins */
int oz_transfer_weights(double theta, int quadratic, double* wt3, double* prolong_even6, double* prolong_odd6,
                        double* restrict4)
{
    static const double nodes[4] = {-1.5, -0.5, 0.5, 1.5};
    time_weights(theta, quadratic, wt3);
    prolong_1d(0, 0, prolong_even6);
    prolong_1d(1, 0, prolong_odd6);
    lagrange_weights(nodes, 4, 0.0, restrict4);
    return 0;
}

/* probe: the exchange at depth d on the patches' states (mode 0 the
   averaging of overlapping active cells, mode 1 the ghost copy) */
int oz_exchange(oz_level* lv, int np, int depth, int mode, int nthreads)
{
    hierarchy H;
    memset(&H, 0, sizeof(H));
    if (!lv || np < 1 || np > OZ_MAXPATCH || (mode != 0 && mode != 1)) return -1;
    H.lv = lv;
    H.np = np;
    H.nt = nthreads < 1 ? 1 : nthreads;
    if (hier_geometry(&H)) return -1;
    double* arr[OZ_MAXPATCH];
    for (int q = 0; q < np; ++q) arr[q] = lv[q].u;
    if (mode == 0)
        exchange_average(&H, depth, arr);
    else
        exchange_ghosts(&H, depth, arr);
    return 0;
}


/* ------------------------------------------------------------------ */
/* Moving levels (Sec. 2.2.1): each tracked object (a puncture) moves   */
/* with dx^i/dt = -beta^i, beta interpolated at the puncture on the     */
/* object's finest patch; after each root step every moving patch whose */
/* centre is more than two of its cells from its object's puncture (per */
/* direction) shifts by two of its cells -- one parent cell, so parent  */
/* and child cell faces stay aligned -- toward it; its cells that were  */
/* already covered keep their values, newly covered ones are prolonged  */
/* from the parent.                                                     */
/* Readings: Heun's method for the track with beta by 4-point Lagrange  */
/* interpolation in each direction from active cells only; patches are  */
/* shifted in index order (a parent before its children, so new cells   */
/* are prolonged from the shifted parent); the children of a shifted    */
/* patch keep their place in space; after a shift the patch's earlier   */
/* time level is dropped (its children interpolate linearly once).      */
/* ------------------------------------------------------------------ */

/* 4-point Lagrange interpolation of beta at x from patch L (nodes: the
   cell centres i0-1 .. i0+2 around x in each direction, all active; refl:
   z layers below the symmetry plane are mirror images of those above) */
static int interp_beta(const oz_level* L, const double x[3], int refl, double b[3])
{
    static const double nodes[4] = {-1.0, 0.0, 1.0, 2.0};
    grid g;
    make_level_grid(&g, L, BC_COPY);
    double w[3][4];
    int lo[3];
    for (int d = 0; d < 3; ++d) {
        const double sc = (x[d] - L->x0[d]) / L->h[d]; /* active-index coordinate */
        const int i0 = (int)floor(sc);
        const int reach = (d == 2 && refl) ? -L->n[d] : 0; /* lowest active index the stencil may use */
        if (!(sc > -2.0 + reach && sc < L->n[d] + 1.0) || i0 - 1 < reach || i0 + 2 >= L->n[d]) return -1;
        lo[d] = i0 - 1 + L->ng;
        lagrange_weights(nodes, 4, sc - i0, w[d]);
    }
    for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int k = 0; k < 4; ++k) {
            int kz = lo[2] + k;
            double sg = 1.0;
            if (kz < L->ng) { /* only with refl: mirrored layer */
                kz = 2 * L->ng - 1 - kz;
                sg = z_parity(IBE + a);
            }
            for (int j = 0; j < 4; ++j)
                for (int i = 0; i < 4; ++i)
                    s += w[2][k] * w[1][j] * w[0][i] * (sg * L->u[(IBE + a) * L->sf + lin(&g, lo[0] + i, lo[1] + j, kz)]);
        }
        b[a] = s;
    }
    return 0;
}

/* shift of patch L toward the puncture xp: -1, 0 or +1 parent cells per direction */
static int patch_shift(const oz_level* L, const double xp[3], int sh[3])
{
    int any = 0;
    for (int d = 0; d < 3; ++d) {
        const double c = L->x0[d] + 0.5 * (L->n[d] - 1) * L->h[d];
        sh[d] = xp[d] - c > 2.0 * L->h[d] ? 1 : (xp[d] - c < -2.0 * L->h[d] ? -1 : 0);
        any |= sh[d] != 0;
    }
    return any;
}

static int regrid(hierarchy* H)
{
    oz_level* lv = H->lv;
    for (int q = 1; q < H->np; ++q) {
        oz_level* L = &lv[q];
        if (L->obj < 0 || L->obj >= H->nobj) continue;
        const oz_level* P = &lv[L->parent];
        int sh[3];
        patch_shift(L, H->xp + 3 * L->obj, sh);
        if (H->plane[q]) sh[2] = 0; /* a patch on the symmetry plane stays on it */
        if (!sh[0] && !sh[1] && !sh[2]) continue;
        grid g, gp;
        make_level_grid(&g, L, BC_COPY);
        make_level_grid(&gp, P, BC_COPY);
        const size_t bytes = (size_t)NF * (size_t)L->sf * sizeof(double);
        double* nu = malloc(bytes);
        if (!nu) return -3;
        memcpy(nu, L->u, bytes);
        int F[3];
        for (int d = 0; d < 3; ++d) F[d] = L->F[d] + sh[d];
#pragma omp parallel for schedule(static) num_threads(H->nt)
        for (int k = 0; k < L->n[2]; ++k)
            for (int j = 0; j < L->n[1]; ++j)
                for (int i = 0; i < L->n[0]; ++i) {
                    const int a[3] = {i, j, k};
                    int src[3], inside = 1;
                    for (int d = 0; d < 3; ++d) {
                        src[d] = a[d] + 2 * sh[d];
                        inside &= src[d] >= 0 && src[d] < L->n[d];
                    }
                    const long x = lin(&g, i + L->ng, j + L->ng, k + L->ng);
                    if (inside) {
                        const long xs = lin(&g, src[0] + L->ng, src[1] + L->ng, src[2] + L->ng);
                        for (int f = 0; f < NF; ++f) nu[f * L->sf + x] = L->u[f * L->sf + xs];
                        continue;
                    }
                    double wx[6], wy[6], wz[6];
                    const int lx = prolong_1d(i, F[0], wx) + P->ng;
                    const int ly = prolong_1d(j, F[1], wy) + P->ng;
                    const int lz = prolong_1d(k, F[2], wz) + P->ng;
                    for (int f = 0; f < NF; ++f) {
                        double s = 0.0;
                        for (int c = 0; c < 6; ++c) {
                            int kz = lz + c;
                            double sg = 1.0;
                            if (H->plane[q] && kz < P->ng) {
                                kz = 2 * P->ng - 1 - kz;
                                sg = z_parity(f);
                            }
                            for (int b = 0; b < 6; ++b)
                                for (int m = 0; m < 6; ++m)
                                    s += wz[c] * wy[b] * wx[m] * (sg * P->u[f * P->sf + lin(&gp, lx + m, ly + b, kz)]);
                        }
                        nu[f * L->sf + x] = s;
                    }
                }
        memcpy(L->u, nu, bytes);
        free(nu);
        for (int d = 0; d < 3; ++d) {
            L->F[d] = F[d];
            L->x0[d] += 2.0 * sh[d] * L->h[d];
        }
        for (int c = q + 1; c < H->np; ++c)
            if (lv[c].parent == q)
                for (int d = 0; d < 3; ++d) lv[c].F[d] -= 2 * sh[d];
        L->has_prev = 0;
        /* a shifted parent's new cells must be in place before its children use them */
        if (hier_geometry(H)) return -4;
    }
    return hier_geometry(H) ? -4 : 0;
}

/* Advance a hierarchy whose patches with obj >= 0 follow the punctures xp
   (3 per object, in/out): per root step, the subcycled step with tracking,
   then the regrid. */
int oz_bo_advance_moving(oz_level* lv, int np, int nobj, double* xp, const oz_params* p, double dt0, int nsteps,
                         int nthreads)
{
    hierarchy H;
    if (!xp || nobj < 1 || !p || !(dt0 > 0) || nsteps < 0) return -1;
    int rc = hier_init(&H, lv, np, p, dt0, nobj, xp, nthreads);
    if (rc) return rc;
    for (int s = 0; s < nsteps && !rc; ++s) {
        rc = bo_depth(&H, 0, 0.0);
        if (!rc) rc = regrid(&H);
    }
    hier_release(&H);
    return rc;
}

/* probe: 4-point Lagrange interpolation of the shift of one patch at x */
int oz_interp_beta(const double* u, long sf, const int* n, int ng, const double* h, const double* x0, const double* x,
                   double* b)
{
    if (!u || !n || !h || !x0 || !x || !b) return -1;
    oz_level L;
    memset(&L, 0, sizeof(L));
    L.u = (double*)u;
    L.prev = (double*)u;
    L.sf = sf;
    L.ng = ng;
    for (int d = 0; d < 3; ++d) {
        L.n[d] = n[d];
        L.h[d] = h[d];
        L.x0[d] = x0[d];
    }
    return interp_beta(&L, x, 0, b);
}

/* probe: one regrid of the moving patches toward xp (no time step) */
int oz_regrid(oz_level* lv, int np, int nobj, double* xp, int nthreads)
{
    hierarchy H;
    if (!xp || nobj < 1) return -1;
    int rc = hier_init(&H, lv, np, NULL, 1.0, nobj, xp, nthreads);
    if (rc) return rc;
    rc = regrid(&H);
    hier_release(&H);
    return rc;
}
