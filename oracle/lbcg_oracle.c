/*
 * lbcg_oracle.c -- plain FP64 CPU oracle of the improved three-dimensional
 * color-gradient lattice Boltzmann model (Wen, Li, Yu & Luo, arXiv 1904.03618).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, literal reference that the
 * GPU path is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product library never
 * does.  It shares no code, header, table or constant with the GPU path.
 *
 * Everything is written in the paper's order and notation, per colour k in
 * {R, B}, with dense 19x19 matrices:
 *   - D3Q19 velocities e_i and weights w_i ............ Eq. (5), text after Eq. (6)
 *   - pressure weights phi_i^k ......................... Eq. (13)
 *   - improved equilibrium f^{k,eq} .................... Eq. (18) (coefficient read
 *     as 3, so that its third moments are the ones Eq. (19) and the Appendix print)
 *   - original equilibrium (improved = 0) .............. Eq. (6)
 *   - macroscopic moments .............................. Eq. (4)
 *   - phase field rho^N and perturbation ............... Eq. (8)
 *   - correction term C^k, Q_alpha, gradient stencil ... Eq. (45)-(49)
 *   - MRT collision in moment space .................... Eq. (40)-(44), Appendix M
 *   - tau_v interpolation across the interface ......... Eq. (52)
 *   - tau-independent perturbation Lambda*Omega2 ....... Eq. (53)
 *   - recoloring ....................................... Eq. (10)-(12)
 *   - streaming ........................................ text after Eq. (12)
 * Readings where the paper is silent (body force, wetting ghost layer, the
 * parabolas of Eq. (52), zero colour gradient, halfway bounce-back walls,
 * moving walls) are listed where they are used.
 *
 * Layout: populations f[(k*19 + i)*N + node], node = x + nx*(y + ny*z).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define Q 19

/* Eq. (5): the D3Q19 velocity set, columns i = 0..18, c = 1. */
static const int EX[Q] = {0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0};
static const int EY[Q] = {0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1};
static const int EZ[Q] = {0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1};

typedef struct {
    int nx, ny, nz;
    int bc[3];              /* per axis: 0 periodic, 1 wall (halfway bounce-back) */
    double theta_deg[2];    /* contact angle (through red) at the low / high wall */
    double rho_in[2];       /* rho_R^in, rho_B^in (Eq. 8) */
    double alpha[2];        /* alpha_R, alpha_B (Eq. 13) */
    double tau_v[2];        /* tau_v^R, tau_v^B (Eq. 52) */
    double A[2];            /* A_R, A_B (Eq. 8) */
    double beta;            /* recoloring parameter (Eq. 10-11) */
    double delta;           /* interface half-width of Eq. (52) */
    double tau_e, tau_q, tau_pi;   /* Eq. (44) */
    double force[3];        /* uniform body-force density */
    double grav[3];         /* buoyancy: F += (rho - rho_ref) * grav */
    double rho_ref;
    int improved;           /* 1: Eq. (18) + correction term; 0: Eq. (6), no correction */
    int meq4;               /* rows 16-18 of m^eq: 0 = M f^eq (default), 1 = the Appendix as printed */
    double wall_u[2][3];    /* velocity of the low / high wall of the wall axis (tangential) */
} orc_params;

/* ------------------------------------------------------------------ tables */
static double W[Q], BI[Q], MM[Q][Q], MI[Q][Q];
static int OPP[Q];
static int tables_ready = 0;

/* Gauss-Jordan inversion with partial pivoting (M^-1 is obtained numerically,
 * never typed in, so that it cannot share a typo with anything else). */
static int invert19(double a[Q][Q], double inv[Q][Q])
{
    double m[Q][2 * Q];
    for (int r = 0; r < Q; ++r)
        for (int c = 0; c < 2 * Q; ++c)
            m[r][c] = c < Q ? a[r][c] : (c - Q == r ? 1.0 : 0.0);
    for (int c = 0; c < Q; ++c) {
        int p = c;
        for (int r = c + 1; r < Q; ++r)
            if (fabs(m[r][c]) > fabs(m[p][c])) p = r;
        if (fabs(m[p][c]) < 1e-14) return -1;
        if (p != c)
            for (int k = 0; k < 2 * Q; ++k) { double t = m[c][k]; m[c][k] = m[p][k]; m[p][k] = t; }
        double d = m[c][c];
        for (int k = 0; k < 2 * Q; ++k) m[c][k] /= d;
        for (int r = 0; r < Q; ++r) {
            if (r == c || m[r][c] == 0.0) continue;
            double s = m[r][c];
            for (int k = 0; k < 2 * Q; ++k) m[r][k] -= s * m[c][k];
        }
    }
    for (int r = 0; r < Q; ++r)
        for (int c = 0; c < Q; ++c) inv[r][c] = m[r][c + Q];
    return 0;
}

static void build_tables(void)
{
    if (tables_ready) return;
    for (int i = 0; i < Q; ++i) {
        int e2 = EX[i] * EX[i] + EY[i] * EY[i] + EZ[i] * EZ[i];
        /* weights w_i (text after Eq. 6) and B_i (text after Eq. 8) */
        W[i] = e2 == 0 ? 1.0 / 3.0 : (e2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
        BI[i] = e2 == 0 ? -1.0 / 3.0 : (e2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0);
        for (int j = 0; j < Q; ++j)
            if (EX[j] == -EX[i] && EY[j] == -EY[i] && EZ[j] == -EZ[i]) OPP[i] = j;
        /* Eq. (43): the 19 raw-moment rows of M */
        double x = EX[i], y = EY[i], z = EZ[i];
        double row[Q] = {1.0, x, y, z, x * x + y * y + z * z,
                         2 * x * x - y * y - z * z, y * y - z * z,
                         x * y, x * z, y * z,
                         x * x * y, x * y * y, x * x * z, x * z * z, y * y * z, y * z * z,
                         x * x * y * y, x * x * z * z, y * y * z * z};
        for (int r = 0; r < Q; ++r) MM[r][i] = row[r];
    }
    invert19(MM, MI);
    tables_ready = 1;
}

static void matvec(double m[Q][Q], const double *v, double *out)
{
    for (int r = 0; r < Q; ++r) {
        double s = 0.0;
        for (int c = 0; c < Q; ++c) s += m[r][c] * v[c];
        out[r] = s;
    }
}

/* Eq. (13): pressure weights of colour k. */
static double phi_k(const orc_params *p, int k, int i)
{
    int e2 = EX[i] * EX[i] + EY[i] * EY[i] + EZ[i] * EZ[i];
    double a = p->alpha[k];
    return e2 == 0 ? a : (e2 == 1 ? (1.0 - a) / 12.0 : (1.0 - a) / 24.0);
}

/* (c_s^k)^2 = (1 - alpha_k)/2, text after Eq. (13). */
static double cs2_k(const orc_params *p, int k) { return 0.5 * (1.0 - p->alpha[k]); }

/* Eq. (18) (improved) or Eq. (6) (original); c = 1. */
static void feq_k(const orc_params *p, int k, double rho, const double u[3], double *out)
{
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double cs2 = cs2_k(p, k);
    for (int i = 0; i < Q; ++i) {
        double eu = EX[i] * u[0] + EY[i] * u[1] + EZ[i] * u[2];
        double e2 = EX[i] * EX[i] + EY[i] * EY[i] + EZ[i] * EZ[i];
        double br = 3.0 * eu + 4.5 * eu * eu - 1.5 * uu;
        if (p->improved)
            br += 3.0 * eu * (3.0 * cs2 - 1.0) * (3.0 * e2 - 5.0);
        out[i] = rho * (phi_k(p, k, i) + W[i] * br);
    }
}

/* ------------------------------------------------------------ exported API */
void orc_tables(double *e, double *w, double *b, int *opp, double *m, double *minv)
{
    build_tables();
    for (int i = 0; i < Q; ++i) {
        if (e) { e[3 * i] = EX[i]; e[3 * i + 1] = EY[i]; e[3 * i + 2] = EZ[i]; }
        if (w) w[i] = W[i];
        if (b) b[i] = BI[i];
        if (opp) opp[i] = OPP[i];
    }
    for (int r = 0; r < Q; ++r)
        for (int c = 0; c < Q; ++c) {
            if (m) m[r * Q + c] = MM[r][c];
            if (minv) minv[r * Q + c] = MI[r][c];
        }
}

void orc_feq(const orc_params *p, int k, double rho, const double *u, double *out)
{
    build_tables();
    feq_k(p, k, rho, u, out);
}

/* Eq. (52); the parabolas g^R, g^B are not printed in the paper.  Reading:
 * the usual quadratic pair that equals the harmonic mean 2 tR tB/(tR+tB) at
 * rho^N = 0 and joins tau_v^R (tau_v^B) with zero slope at +delta (-delta). */
double orc_tau_v(const orc_params *p, double rhoN)
{
    double tR = p->tau_v[0], tB = p->tau_v[1], d = p->delta;
    if (rhoN > d) return tR;
    if (rhoN < -d) return tB;
    double s1 = 2.0 * tR * tB / (tR + tB);
    if (rhoN > 0.0) {
        double s2 = 2.0 * (tR - s1) / d, s3 = -s2 / (2.0 * d);
        return s1 + s2 * rhoN + s3 * rhoN * rhoN;
    }
    double t2 = 2.0 * (s1 - tB) / d, t3 = t2 / (2.0 * d);
    return s1 + t2 * rhoN + t3 * rhoN * rhoN;
}

/* Relaxation rates of Eq. (44). */
static void s_diag(const orc_params *p, double tau_v, double *s)
{
    for (int r = 0; r < 4; ++r) s[r] = 1.0;
    s[4] = 1.0 / p->tau_e;
    for (int r = 5; r < 10; ++r) s[r] = 1.0 / tau_v;
    for (int r = 10; r < 16; ++r) s[r] = 1.0 / p->tau_q;
    for (int r = 16; r < 19; ++r) s[r] = 1.0 / p->tau_pi;
}

/*
 * Collision of one colour at one node: Eq. (12) with Omega1 from Eq. (41)-(42)
 * and Omega2 from Eq. (8) rescaled by Eq. (53).
 *   f      : f^k at the node (19)
 *   rho_k  : colour density, rho: total density, u: mixture velocity
 *   grad   : colour gradient grad(rho^N) (Eq. 49 stencil)
 *   Qk     : Q_x, Q_y, Q_z of colour k (Eq. 46-49)
 *   F      : total body-force density at the node (reading: Guo forcing, the
 *            colour share is (rho_k/rho) F, added as (I - S/2) M F^Guo)
 *   out    : f^{*,k} (19)
 */
void orc_collide_color(const orc_params *p, int k, const double *f, double rho_k, double rho,
                       const double *u, double tau_v, const double *grad, const double *Qk,
                       const double *F, double *out)
{
    build_tables();
    double s[Q], m[Q], feq[Q], meq[Q], C[Q], gu[Q], mF[Q], mbar[Q], om1[Q];
    s_diag(p, tau_v, s);
    matvec(MM, f, m);
    feq_k(p, k, rho_k, u, feq);
    matvec(MM, feq, meq);                       /* m^{k,eq} = M f^{k,eq} (after Eq. 53/44) */
    if (p->meq4) {
        /* The Appendix prints rows 16-18 of m^{k,eq} with 2 rho_k c^2 (u_a^2 + u_b^2)
         * where M f^{k,eq} gives 3 rho_k (u_a^2 + u_b^2); this switch takes the
         * printed rows instead of M f^eq (c = 1). */
        double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
        double base = rho_k * (1.0 - p->alpha[k] - uu);
        meq[16] = (base + 2.0 * rho_k * (u[0] * u[0] + u[1] * u[1])) / 6.0;
        meq[17] = (base + 2.0 * rho_k * (u[0] * u[0] + u[2] * u[2])) / 6.0;
        meq[18] = (base + 2.0 * rho_k * (u[1] * u[1] + u[2] * u[2])) / 6.0;
    }
    for (int r = 0; r < Q; ++r) C[r] = 0.0;
    if (p->improved) {                          /* Eq. (45) */
        C[4] = Qk[0] + Qk[1] + Qk[2];
        C[5] = 2.0 * Qk[0] - Qk[1] - Qk[2];
        C[6] = Qk[1] - Qk[2];
    }
    /* body force: Guo's source of the colour share F_k = (rho_k/rho) F */
    double Fk[3] = {F[0] * rho_k / rho, F[1] * rho_k / rho, F[2] * rho_k / rho};
    for (int i = 0; i < Q; ++i) {
        double eu = EX[i] * u[0] + EY[i] * u[1] + EZ[i] * u[2];
        double eF = EX[i] * Fk[0] + EY[i] * Fk[1] + EZ[i] * Fk[2];
        double uF = u[0] * Fk[0] + u[1] * Fk[1] + u[2] * Fk[2];
        gu[i] = W[i] * (3.0 * (eF - uF) + 9.0 * eu * eF);
    }
    matvec(MM, gu, mF);
    for (int r = 0; r < Q; ++r)                 /* Eq. (41) (+ force) */
        mbar[r] = -s[r] * (m[r] - meq[r]) + (1.0 - 0.5 * s[r]) * (C[r] + mF[r]);
    matvec(MI, mbar, om1);                      /* Eq. (42) */

    /* Eq. (8); a zero gradient gives no perturbation (the direction is undefined). */
    double g = sqrt(grad[0] * grad[0] + grad[1] * grad[1] + grad[2] * grad[2]);
    double om2[Q], mo2[Q], om2n[Q];
    for (int i = 0; i < Q; ++i) om2[i] = 0.0;
    if (g > 1e-12) {
        for (int i = 0; i < Q; ++i) {
            double eg = EX[i] * grad[0] + EY[i] * grad[1] + EZ[i] * grad[2];
            om2[i] = 0.5 * p->A[k] * g * (W[i] * eg * eg / (g * g) - BI[i]);
        }
    }
    matvec(MM, om2, mo2);                       /* Eq. (53): Lambda = M^-1 S M */
    for (int r = 0; r < Q; ++r) mo2[r] *= s[r];
    matvec(MI, mo2, om2n);
    for (int i = 0; i < Q; ++i) out[i] = f[i] + om1[i] + om2n[i];   /* Eq. (12) */
}

/* Eq. (10)-(11) at one node.  fstar is the post-perturbation total f*. */
void orc_recolor(const orc_params *p, const double *fstar, double rhoR, double rhoB,
                 const double *grad, double *outR, double *outB)
{
    build_tables();
    double rho = rhoR + rhoB;
    double g = sqrt(grad[0] * grad[0] + grad[1] * grad[1] + grad[2] * grad[2]);
    for (int i = 0; i < Q; ++i) {
        /* sum_k f^{k,eq}(rho_k, alpha_k, u = 0) = sum_k rho_k phi_i^k */
        double f0 = rhoR * phi_k(p, 0, i) + rhoB * phi_k(p, 1, i);
        double cosv = 0.0;
        double en = sqrt((double)(EX[i] * EX[i] + EY[i] * EY[i] + EZ[i] * EZ[i]));
        if (i != 0 && g > 1e-12)
            cosv = (EX[i] * grad[0] + EY[i] * grad[1] + EZ[i] * grad[2]) / (en * g);
        double seg = p->beta * rhoR * rhoB / (rho * rho) * cosv * f0;
        outR[i] = rhoR / rho * fstar[i] + seg;
        outB[i] = rhoB / rho * fstar[i] - seg;
    }
}

/* -------------------------------------------------------------- lattice */
typedef struct {
    const orc_params *p;
    int64_t N;
    int wall;            /* wall axis, or -1 */
    int n[3];
} lat_t;

static void lat_init(lat_t *L, const orc_params *p)
{
    L->p = p;
    L->n[0] = p->nx; L->n[1] = p->ny; L->n[2] = p->nz;
    L->N = (int64_t)p->nx * p->ny * p->nz;
    L->wall = -1;
    for (int a = 0; a < 3; ++a) if (p->bc[a]) L->wall = a;
}

static int64_t idx(const lat_t *L, const int c[3])
{
    return (int64_t)c[0] + (int64_t)L->n[0] * ((int64_t)c[1] + (int64_t)L->n[1] * c[2]);
}

static int wrap(int v, int n) { v %= n; return v < 0 ? v + n : v; }

/* Body-force density at a node: uniform part plus buoyancy (reading). */
static void body_force(const orc_params *p, double rho, double *F)
{
    for (int a = 0; a < 3; ++a) F[a] = p->force[a] + (rho - p->rho_ref) * p->grav[a];
}

/* Eq. (4) at one node; u carries half the body force (Guo reading). */
static void node_macro(const lat_t *L, const double *f, int64_t node,
                       double *rhoR, double *rhoB, double *u, double *F)
{
    double r[2] = {0.0, 0.0}, j[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < 2; ++k)
        for (int i = 0; i < Q; ++i) {
            double v = f[(int64_t)(k * Q + i) * L->N + node];
            r[k] += v;
            j[0] += EX[i] * v; j[1] += EY[i] * v; j[2] += EZ[i] * v;
        }
    double rho = r[0] + r[1];
    body_force(L->p, rho, F);
    for (int a = 0; a < 3; ++a) u[a] = (j[a] + 0.5 * F[a]) / rho;
    *rhoR = r[0]; *rhoB = r[1];
}

/* Field value at c + d, where c + d may sit one layer beyond a wall: then the
 * ghost plane value is returned (ghost planes are indexed by the node of the
 * first fluid layer they face). */
static double field_at(const lat_t *L, const double *fld, const double *glo, const double *ghi,
                       const int c[3], const int d[3], int stride, int comp)
{
    int q[3];
    int side = 0;
    for (int a = 0; a < 3; ++a) {
        int v = c[a] + d[a];
        if (a == L->wall && (v < 0 || v >= L->n[a])) {
            side = v < 0 ? -1 : 1;
            v = v < 0 ? 0 : L->n[a] - 1;
        } else {
            v = wrap(v, L->n[a]);
        }
        q[a] = v;
    }
    int64_t node = idx(L, q);
    if (side == 0) return fld[node * stride + comp];
    return (side < 0 ? glo : ghi)[node * stride + comp];
}

/* Eq. (49): isotropic gradient 3 sum_i w_i psi(x + e_i) e_i of component
 * `comp` of a field stored with `stride` values per node. */
static void iso_grad(const lat_t *L, const double *fld, const double *glo, const double *ghi,
                     const int c[3], int stride, int comp, double *g)
{
    g[0] = g[1] = g[2] = 0.0;
    for (int i = 1; i < Q; ++i) {
        int d[3] = {EX[i], EY[i], EZ[i]};
        double v = field_at(L, fld, glo, ghi, c, d, stride, comp);
        g[0] += 3.0 * W[i] * v * EX[i];
        g[1] += 3.0 * W[i] * v * EY[i];
        g[2] += 3.0 * W[i] * v * EZ[i];
    }
}

/*
 * Ghost planes one layer beyond each wall (reading; the paper gives no wetting
 * scheme).  For the phase field the geometric rule: the wall-normal difference
 * across the half link equals -cot(theta) times the in-plane gradient
 * magnitude, so that the interface meets the wall at theta (measured through
 * red); theta = 90 deg gives a mirror.  The in-plane gradient is the 2D
 * isotropic stencil (weights 1/9 axis, 1/36 diagonal).  For Qbar (which holds
 * u, zero at the halfway wall) the odd reflection -Qbar of the first layer.
 */
static void build_ghosts(const lat_t *L, const double *rhoN, const double *qbar, const double *rhoR_l,
                         const double *rhoB_l, double *gN_lo, double *gN_hi, double *gQ_lo, double *gQ_hi)
{
    int a = L->wall;
    if (a < 0) return;
    int b = (a + 1) % 3, cax = (a + 2) % 3;
    const orc_params *p = L->p;
    double cot[2];
    for (int s = 0; s < 2; ++s) cot[s] = tan((90.0 - p->theta_deg[s]) * M_PI / 180.0);
    for (int s = 0; s < 2; ++s) {
        int layer = s == 0 ? 0 : L->n[a] - 1;
        double *gN = s == 0 ? gN_lo : gN_hi;
        double *gQ = s == 0 ? gQ_lo : gQ_hi;
        for (int j = 0; j < L->n[cax]; ++j)
            for (int i = 0; i < L->n[b]; ++i) {
                int c[3];
                c[a] = layer; c[b] = i; c[cax] = j;
                int64_t node = idx(L, c);
                double gb = 0.0, gc = 0.0;
                for (int db = -1; db <= 1; ++db)
                    for (int dc = -1; dc <= 1; ++dc) {
                        if (db == 0 && dc == 0) continue;
                        double w2 = (db != 0 && dc != 0) ? 1.0 / 36.0 : 1.0 / 9.0;
                        int q[3];
                        q[a] = layer; q[b] = wrap(i + db, L->n[b]); q[cax] = wrap(j + dc, L->n[cax]);
                        double v = rhoN[idx(L, q)];
                        gb += 3.0 * w2 * v * db;
                        gc += 3.0 * w2 * v * dc;
                    }
                double gpar = sqrt(gb * gb + gc * gc);
                gN[node] = rhoN[node] + cot[s] * gpar;
                /* Qbar^k = rho_k u (1 - 3 cs2_k) takes the wall's value half way:
                 * ghost = 2 Qbar^k(wall) - Qbar^k(first layer), with the wall
                 * velocity and the first layer's colour densities. */
                for (int k = 0; k < 2; ++k) {
                    const double rk = k == 0 ? rhoR_l[node] : rhoB_l[node];
                    const double qc = 1.0 - 1.5 * (1.0 - p->alpha[k]);
                    for (int a3 = 0; a3 < 3; ++a3)
                        gQ[node * 6 + 3 * k + a3] = 2.0 * rk * p->wall_u[s][a3] * qc - qbar[node * 6 + 3 * k + a3];
                }
            }
    }
}

/* Equilibrium initial state: f^k = f^{k,eq}(rho_k, u0). */
void orc_init(const orc_params *p, const double *rhoR0, const double *rhoB0,
              const double *ux0, const double *uy0, const double *uz0, double *f)
{
    build_tables();
    lat_t L; lat_init(&L, p);
    #pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < L.N; ++n) {
        double u[3] = {ux0[n], uy0[n], uz0[n]}, fe[Q];
        const double *r[2] = {rhoR0, rhoB0};
        for (int k = 0; k < 2; ++k) {
            feq_k(p, k, r[k][n], u, fe);
            for (int i = 0; i < Q; ++i) f[(int64_t)(k * Q + i) * L.N + n] = fe[i];
        }
    }
}

/*
 * Per-node fields at the current level: rho^N (Eq. 8 text), the colour
 * gradient and the per-colour Q_alpha (Eq. 46-49).  Any output may be NULL.
 * grad: 3 per node; Q: 6 per node (Q^R_x,y,z, Q^B_x,y,z).
 */
static void stencil_fields(const lat_t *L, const double *f, double *rhoR, double *rhoB,
                           double *u, double *rhoN, double *qbar, double *grad, double *Qk,
                           double *gN_lo, double *gN_hi, double *gQ_lo, double *gQ_hi)
{
    const orc_params *p = L->p;
    #pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < L->N; ++n) {
        double F[3];
        node_macro(L, f, n, &rhoR[n], &rhoB[n], &u[3 * n], F);
        double a = rhoR[n] / p->rho_in[0], b = rhoB[n] / p->rho_in[1];
        rhoN[n] = (a - b) / (a + b);
        const double r[2] = {rhoR[n], rhoB[n]};
        for (int k = 0; k < 2; ++k)
            for (int c = 0; c < 3; ++c)
                qbar[6 * n + 3 * k + c] = r[k] * u[3 * n + c] * (1.0 - 3.0 * cs2_k(p, k));
    }
    build_ghosts(L, rhoN, qbar, rhoR, rhoB, gN_lo, gN_hi, gQ_lo, gQ_hi);
    #pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < L->N; ++n) {
        int c[3] = {(int)(n % L->n[0]), (int)((n / L->n[0]) % L->n[1]), (int)(n / ((int64_t)L->n[0] * L->n[1]))};
        iso_grad(L, rhoN, gN_lo, gN_hi, c, 1, 0, &grad[3 * n]);
        for (int k = 0; k < 2; ++k)
            for (int al = 0; al < 3; ++al) {
                double g3[3];
                iso_grad(L, qbar, gQ_lo, gQ_hi, c, 6, 3 * k + al, g3);
                Qk[6 * n + 3 * k + al] = g3[al];   /* Q_alpha = d_alpha Qbar_alpha */
            }
    }
}

typedef struct {
    double *rhoR, *rhoB, *u, *rhoN, *qbar, *grad, *Qk, *gN_lo, *gN_hi, *gQ_lo, *gQ_hi, *fpost;
} work_t;

static int work_alloc(work_t *w, const lat_t *L)
{
    int64_t N = L->N;
    int64_t plane = 1;
    if (L->wall >= 0) plane = N;   /* ghost planes are indexed by node (simple, oversized) */
    w->rhoR = malloc(sizeof(double) * N);
    w->rhoB = malloc(sizeof(double) * N);
    w->u = malloc(sizeof(double) * 3 * N);
    w->rhoN = malloc(sizeof(double) * N);
    w->qbar = malloc(sizeof(double) * 6 * N);
    w->grad = malloc(sizeof(double) * 3 * N);
    w->Qk = malloc(sizeof(double) * 6 * N);
    w->gN_lo = malloc(sizeof(double) * plane);
    w->gN_hi = malloc(sizeof(double) * plane);
    w->gQ_lo = malloc(sizeof(double) * 6 * plane);
    w->gQ_hi = malloc(sizeof(double) * 6 * plane);
    w->fpost = malloc(sizeof(double) * 2 * Q * N);
    return (w->rhoR && w->rhoB && w->u && w->rhoN && w->qbar && w->grad && w->Qk &&
            w->gN_lo && w->gN_hi && w->gQ_lo && w->gQ_hi && w->fpost) ? 0 : -1;
}

static void work_free(work_t *w)
{
    free(w->rhoR); free(w->rhoB); free(w->u); free(w->rhoN); free(w->qbar); free(w->grad);
    free(w->Qk); free(w->gN_lo); free(w->gN_hi); free(w->gQ_lo); free(w->gQ_hi); free(w->fpost);
}

/* Pull source of direction i at node c: (source node, source direction).
 * Periodic wrap, or halfway bounce-back when x - e_i lies beyond a wall.
 * *side (optional) is -1 without bounce-back, else 0 / 1 for the low / high wall. */
static void pull_source_side(const lat_t *L, const int c[3], int i, int64_t *src, int *dir, int *side)
{
    int e[3] = {EX[i], EY[i], EZ[i]};
    int q[3];
    if (side) *side = -1;
    for (int a = 0; a < 3; ++a) {
        int v = c[a] - e[a];
        if (a == L->wall && (v < 0 || v >= L->n[a])) {
            *src = idx(L, c);
            *dir = OPP[i];
            if (side) *side = v < 0 ? 0 : 1;
            return;
        }
        q[a] = wrap(v, L->n[a]);
    }
    *src = idx(L, q);
    *dir = i;
}

static void pull_source(const lat_t *L, const int c[3], int i, int64_t *src, int *dir)
{
    pull_source_side(L, c, i, src, dir, NULL);
}

/* One time step t -> t+1: collide + perturb + recolor at every node, then stream. */
static void one_step(const lat_t *L, const double *f, double *fnext, work_t *w)
{
    const orc_params *p = L->p;
    const int64_t N = L->N;
    stencil_fields(L, f, w->rhoR, w->rhoB, w->u, w->rhoN, w->qbar, w->grad, w->Qk,
                   w->gN_lo, w->gN_hi, w->gQ_lo, w->gQ_hi);
    #pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        double rho = w->rhoR[n] + w->rhoB[n], F[3];
        body_force(p, rho, F);
        double tau = orc_tau_v(p, w->rhoN[n]);
        double fk[Q], fs[Q], fstar[Q], oR[Q], oB[Q];
        const double rk[2] = {w->rhoR[n], w->rhoB[n]};
        for (int i = 0; i < Q; ++i) fstar[i] = 0.0;
        for (int k = 0; k < 2; ++k) {
            for (int i = 0; i < Q; ++i) fk[i] = f[(int64_t)(k * Q + i) * N + n];
            orc_collide_color(p, k, fk, rk[k], rho, &w->u[3 * n], tau, &w->grad[3 * n],
                              &w->Qk[6 * n + 3 * k], F, fs);
            for (int i = 0; i < Q; ++i) fstar[i] += fs[i];
        }
        orc_recolor(p, fstar, rk[0], rk[1], &w->grad[3 * n], oR, oB);
        for (int i = 0; i < Q; ++i) {
            w->fpost[(int64_t)i * N + n] = oR[i];
            w->fpost[(int64_t)(Q + i) * N + n] = oB[i];
        }
    }
    #pragma omp parallel for schedule(static)
    for (int64_t n = 0; n < N; ++n) {
        int c[3] = {(int)(n % L->n[0]), (int)((n / L->n[0]) % L->n[1]), (int)(n / ((int64_t)L->n[0] * L->n[1]))};
        for (int i = 0; i < Q; ++i) {
            int64_t src; int dir, side;
            pull_source_side(L, c, i, &src, &dir, &side);
            for (int k = 0; k < 2; ++k) {
                double v = w->fpost[(int64_t)(k * Q + dir) * N + src];
                /* Moving halfway wall (reading; the paper uses moving plates in
                 * Sec. IV.A): the reflected population of colour k gains twice
                 * the odd part of the model's own equilibrium (Eq. 18, or Eq. 6
                 * for the original model) at the wall velocity U_w,
                 * f_i^{k,eq}(rho_k, U_w) - f_opp(i)^{k,eq}(rho_k, U_w), with rho_k
                 * this node's colour density.  A uniform flow at U_w is then a
                 * fixed point of the wall. */
                if (side >= 0) {
                    double fw[Q];
                    feq_k(p, k, k == 0 ? w->rhoR[n] : w->rhoB[n], p->wall_u[side], fw);
                    v += fw[i] - fw[OPP[i]];
                }
                fnext[(int64_t)(k * Q + i) * N + n] = v;
            }
        }
    }
}

/* Advance f (in place) by nsteps.  Returns 0, or -1 on allocation failure. */
int orc_run(const orc_params *p, double *f, int64_t nsteps)
{
    build_tables();
    lat_t L; lat_init(&L, p);
    work_t w;
    double *tmp = malloc(sizeof(double) * 2 * Q * L.N);
    if (!tmp || work_alloc(&w, &L)) { free(tmp); return -1; }
    for (int64_t s = 0; s < nsteps; ++s) {
        one_step(&L, f, tmp, &w);
        memcpy(f, tmp, sizeof(double) * 2 * Q * L.N);
    }
    free(tmp);
    work_free(&w);
    return 0;
}

/*
 * Macroscopic fields of the current level (Eq. 4, u with half the force) and
 * the stencil quantities the next collision will use.  Any pointer may be NULL.
 * diag = {sum rho_R, sum rho_B, sum rho u_x, sum rho u_y, sum rho u_z}.
 */
int orc_fields(const orc_params *p, const double *f, double *rhoR, double *rhoB, double *ux,
               double *uy, double *uz, double *rhoN, double *grad, double *Qk, double *diag)
{
    build_tables();
    lat_t L; lat_init(&L, p);
    work_t w;
    if (work_alloc(&w, &L)) return -1;
    stencil_fields(&L, f, w.rhoR, w.rhoB, w.u, w.rhoN, w.qbar, w.grad, w.Qk,
                   w.gN_lo, w.gN_hi, w.gQ_lo, w.gQ_hi);
    double d[5] = {0, 0, 0, 0, 0};
    for (int64_t n = 0; n < L.N; ++n) {
        if (rhoR) rhoR[n] = w.rhoR[n];
        if (rhoB) rhoB[n] = w.rhoB[n];
        if (ux) ux[n] = w.u[3 * n];
        if (uy) uy[n] = w.u[3 * n + 1];
        if (uz) uz[n] = w.u[3 * n + 2];
        if (rhoN) rhoN[n] = w.rhoN[n];
        if (grad) for (int c = 0; c < 3; ++c) grad[3 * n + c] = w.grad[3 * n + c];
        if (Qk) for (int c = 0; c < 6; ++c) Qk[6 * n + c] = w.Qk[6 * n + c];
        double rho = w.rhoR[n] + w.rhoB[n];
        d[0] += w.rhoR[n]; d[1] += w.rhoB[n];
        for (int c = 0; c < 3; ++c) d[2 + c] += rho * w.u[3 * n + c];
    }
    if (diag) for (int c = 0; c < 5; ++c) diag[c] = d[c];
    work_free(&w);
    return 0;
}

/* Streaming/boundary index map: for every (node, i) the pull source. */
void orc_index_map(const orc_params *p, int64_t *src_node, int8_t *src_dir)
{
    build_tables();
    lat_t L; lat_init(&L, p);
    for (int64_t n = 0; n < L.N; ++n) {
        int c[3] = {(int)(n % L.n[0]), (int)((n / L.n[0]) % L.n[1]), (int)(n / ((int64_t)L.n[0] * L.n[1]))};
        for (int i = 0; i < Q; ++i) {
            int64_t s; int d;
            pull_source(&L, c, i, &s, &d);
            src_node[(int64_t)i * L.N + n] = s;
            src_dir[(int64_t)i * L.N + n] = (int8_t)d;
        }
    }
}

/* Number of OpenMP threads the oracle uses (for reporting). */
int orc_threads(void)
{
#ifdef _OPENMP
    extern int omp_get_max_threads(void);
    return omp_get_max_threads();
#else
    return 1;
#endif
}
