/*
 * GRPIC reference oracle: a plain, slow, single-threaded FP64 CPU
 * implementation of one timestep of the general-relativistic PIC cycle of
 * Watson & Nishikawa, "A Method for Incorporating General Relativity in
 * Electromagnetic Particle-in-Cell Code" (arXiv:0904.0232).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads
 * or calls this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark use it.  It shares no code with the HIP
 * path.  Compile with -ffp-contract=off so every product and sum is
 * rounded as written.
 *
 * Units: dx = 1 (node coordinates), x^4 = c t.  Indices are 0-based here:
 * 0,1,2 = x,y,z and 3 = the time component (the paper's index 4).
 *
 * Readings of passages where the paper is silent or garbled are marked
 * "reading:" and are the same as those listed in the design notes.
 *
 * Parity status of each function is stated in its comment.  Pinned means
 * a CPU test checks it against a closed form, a textbook special case,
 * an invariant or brute force; "parity unpinned" means no such check
 * exists and it is trusted only by reading.  Every function is pinned:
 *  - the constitutive step against raising with the metric, pointwise in
 *    Kerr, and its node averaging through Wald's vacuum solution in Kerr,
 *    whose one-cycle change converges at second order;
 *  - the curved face-area weights against a Gauss-Legendre integral of the
 *    metric area density over each sub-rectangle;
 *  - the relaxation layer as the stated pull toward the reference state;
 *  - the field-energy diagnostic against closed-form cavity-mode sums.
 * What the pins do not fix is stated as readings: the inner boundary
 * (excision and relaxation) lets disturbances from inside the horizon out
 * through the centred stencils; Wald's far field stays bounded at about
 * 0.1 B0 rather than at its truncation level.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#define OR_MAXSP 8
#define OR_DEAD 0xFF

typedef struct {
    int32_t nx, ny, nz;
    int32_t gamma_mode;   /* 0: paper's gamma estimate f(u4,a4); 1: gamma = u4/c */
    int32_t deposit_mode; /* 0: curved face-area weights; 1: flat weights       */
    int32_t nspecies;
    int32_t field_iters;  /* evaluations of the constitutive map per half-cycle  */
    int32_t rk_mode;      /* 0: classic RK4 reading; 1: the printed steps        */
    int32_t gather_mode;  /* 0: fields at every stage; 1: at x_n for all stages  */
    int32_t gather_weights; /* 0: trilinear (4-volume, det g = -1); 1: spatial volume */
    double c, dt;
    double m, a;          /* hole mass and spin parameter, in cells              */
    double center[3];     /* hole position in node coordinates                   */
    double r_rm;          /* particles with r below this are removed             */
    double r_exc;         /* field points with r below this are excised          */
    double r_damp;        /* fields are relaxed to their initial values below r  */
    double damp_max;      /* relaxation fraction per step at r = r_exc           */
    double outer_layer;   /* width in cells of the outer absorbing layer (0: off) */
    double outer_damp;    /* its relaxation fraction per step at the outer face  */
    double charge[OR_MAXSP]; /* macro-particle charge per species                */
    double mass[OR_MAXSP];   /* macro-particle mass per species                  */
} or_params;

typedef struct {
    int64_t n_alive[OR_MAXSP];
    int64_t n_removed_horizon;
    int64_t n_removed_outer;
    int64_t gamma_clamps;
    int64_t flags;
    double charge_total;
    double energy_particles;
    double lz_particles;
    double energy_field;
    double gauss_residual_max;
    double mass_shell_residual_max;
} or_diag;

/* ------------------------------------------------------------------ */
/* Metric: Kerr in Cartesian Kerr-Schild form (Sec. 2.1, eq. kerr_metric,
 * the one-form k and eq. radius_eqn).                                 */
/* ------------------------------------------------------------------ */

/* Radius r from r^4 - (R^2 - a^2) r^2 - a^2 z^2 = 0 (eq. radius_eqn).
 * reading: the non-negative root for r^2 of this quadratic in r^2, written
 * in the cancellation-free form on each side of R^2 = a^2.
 * Pinned: quartic residual and the special cases a=0, z=0, x=y=0. */
double or_radius(double a, double x, double y, double z)
{
    double R2 = x * x + y * y + z * z;
    double b = R2 - a * a;
    double s = sqrt(b * b + 4.0 * a * a * z * z);
    double r2;
    if (b >= 0.0)
        r2 = 0.5 * (b + s);
    else
        r2 = (2.0 * a * a * z * z) / (s - b);
    return sqrt(r2);
}

/* The scalar f = 2 m r^3 / (r^4 + a^2 z^2) and the covariant null one-form
 * k_mu = ((r x - a y)/(r^2+a^2), (r y + a x)/(r^2+a^2), z/r, 1) read off the
 * coefficients of dx, dy, dz and dx^4 = c dt in the expression for k
 * (Sec. 2.1).  reading: the "dt" in k is dx^4 = c dt, so k_4 = 1. */
static void ks_fk(const or_params *p, double x, double y, double z,
                  double *r_out, double *f_out, double k[4])
{
    double a = p->a, m = p->m;
    double r = or_radius(a, x, y, z);
    if (m == 0.0) { /* flat space: f = 0 everywhere, including r = 0 */
        k[0] = k[1] = k[2] = 0.0;
        k[3] = 1.0;
        *f_out = 0.0;
        *r_out = r;
        return;
    }
    double rr = r * r;
    double den = rr + a * a;
    double S4 = rr * rr + a * a * z * z;
    k[0] = (r * x - a * y) / den;
    k[1] = (r * y + a * x) / den;
    k[2] = z / r;
    k[3] = 1.0;
    *f_out = 2.0 * m * r * rr / S4;
    *r_out = r;
}

static const double ETA[4] = {1.0, 1.0, 1.0, -1.0};

/* g_{mu nu} = eta + f k_mu k_nu and its inverse.  The inverse is computed
 * here by plain Gauss-Jordan elimination of g (no use of the Kerr-Schild
 * structure), so it is the definition of an inverse written out.
 * Pinned: det g = -1, g g^-1 = I, textbook Schwarzschild form at a=0,
 * Boyer-Lindquist g_tt, g_tphi, g_phiphi and the horizon condition. */
static int invert4(const double A[4][4], double Ainv[4][4])
{
    double M[4][8];
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            M[i][j] = A[i][j];
            M[i][j + 4] = (i == j) ? 1.0 : 0.0;
        }
    for (int col = 0; col < 4; col++) {
        int piv = col;
        for (int i = col + 1; i < 4; i++)
            if (fabs(M[i][col]) > fabs(M[piv][col])) piv = i;
        if (M[piv][col] == 0.0) return -1;
        if (piv != col)
            for (int j = 0; j < 8; j++) {
                double t = M[col][j];
                M[col][j] = M[piv][j];
                M[piv][j] = t;
            }
        double d = M[col][col];
        for (int j = 0; j < 8; j++) M[col][j] /= d;
        for (int i = 0; i < 4; i++) {
            if (i == col) continue;
            double fct = M[i][col];
            if (fct == 0.0) continue;
            for (int j = 0; j < 8; j++) M[i][j] -= fct * M[col][j];
        }
    }
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) Ainv[i][j] = M[i][j + 4];
    return 0;
}

void or_metric(const or_params *p, double x, double y, double z,
               double g[16], double gi[16], double *r_out)
{
    double r, f, k[4];
    ks_fk(p, x, y, z, &r, &f, k);
    double G[4][4], Gi[4][4];
    for (int mu = 0; mu < 4; mu++)
        for (int nu = 0; nu < 4; nu++)
            G[mu][nu] = (mu == nu ? ETA[mu] : 0.0) + f * k[mu] * k[nu];
    invert4((const double(*)[4])G, Gi);
    for (int mu = 0; mu < 4; mu++)
        for (int nu = 0; nu < 4; nu++) {
            g[mu * 4 + nu] = G[mu][nu];
            if (gi) gi[mu * 4 + nu] = Gi[mu][nu];
        }
    if (r_out) *r_out = r;
}

/* Spatial derivatives d_i g_{mu nu} (i = 0..2); the metric is stationary
 * so d_4 g = 0.  Written out from g = eta + f k k with the implicit
 * derivative of eq. radius_eqn:
 *   d_x r = x r^3/(r^4+a^2 z^2), d_y r = y r^3/(r^4+a^2 z^2),
 *   d_z r = z r (r^2+a^2)/(r^4+a^2 z^2).
 * dg[i*16 + mu*4 + nu].  Pinned: against a Richardson-extrapolated
 * central difference of or_metric. */
void or_metric_deriv(const or_params *p, double x, double y, double z, double dg[48])
{
    double a = p->a;
    if (p->m == 0.0) {
        for (int i = 0; i < 48; i++) dg[i] = 0.0;
        return;
    }
    double r, f, k[4];
    ks_fk(p, x, y, z, &r, &f, k);
    double rr = r * r;
    double den = rr + a * a;
    double S4 = rr * rr + a * a * z * z;
    double dr[3];
    dr[0] = x * r * rr / S4;
    dr[1] = y * r * rr / S4;
    dr[2] = z * r * (rr + a * a) / S4;
    double df[3], dk[3][4];
    for (int i = 0; i < 3; i++) {
        double dS4 = 4.0 * rr * r * dr[i] + (i == 2 ? 2.0 * a * a * z : 0.0);
        df[i] = f * (3.0 * dr[i] / r - dS4 / S4);
        double dden = 2.0 * r * dr[i];
        double n0 = dr[i] * x + (i == 0 ? r : 0.0) - (i == 1 ? a : 0.0);
        double n1 = dr[i] * y + (i == 1 ? r : 0.0) + (i == 0 ? a : 0.0);
        dk[i][0] = (n0 - k[0] * dden) / den;
        dk[i][1] = (n1 - k[1] * dden) / den;
        dk[i][2] = ((i == 2 ? 1.0 : 0.0) - k[2] * dr[i]) / r;
        dk[i][3] = 0.0;
    }
    for (int i = 0; i < 3; i++)
        for (int mu = 0; mu < 4; mu++)
            for (int nu = 0; nu < 4; nu++)
                dg[i * 16 + mu * 4 + nu] =
                    df[i] * k[mu] * k[nu] + f * (dk[i][mu] * k[nu] + k[mu] * dk[i][nu]);
}

/* Christoffel symbols of the second kind (Sec. 2.1, eq. Maxwell_Newton:c)
 * by the textbook formula
 *   Gamma^a_{bc} = 1/2 g^{ad} (d_b g_{dc} + d_c g_{db} - d_d g_{bc}),
 * as a full 4x4x4 array G[a*16 + b*4 + c].
 * Pinned: contracted symbol Gamma^b_{bc} = 0 (det g = -1), geodesic
 * conservation of E, L_z and the Carter constant, circular orbits. */
void or_christoffel(const or_params *p, double x, double y, double z, double G[64])
{
    double g[16], gi[16], dg[48];
    or_metric(p, x, y, z, g, gi, NULL);
    or_metric_deriv(p, x, y, z, dg);
#define DG(i, mu, nu) ((i) < 3 ? dg[(i) * 16 + (mu) * 4 + (nu)] : 0.0)
    for (int a = 0; a < 4; a++)
        for (int b = 0; b < 4; b++)
            for (int c = 0; c < 4; c++) {
                double s = 0.0;
                for (int d = 0; d < 4; d++)
                    s += gi[a * 4 + d] * (DG(b, d, c) + DG(c, d, b) - DG(d, b, c));
                G[a * 16 + b * 4 + c] = 0.5 * s;
            }
#undef DG
}

/* ------------------------------------------------------------------ */
/* Grid layout.  Every field component lives on an (nx+3)(ny+3)(nz+3)
 * array; index (i,j,k) with i in [-1, nx+1] maps to offset
 * ((k+1)(ny+3) + (j+1))(nx+3) + (i+1).  A component staggered by +1/2 along
 * an axis stores the point i+1/2 at index i.
 *
 * Yee placement (Sec. 3, the magnetic and electric shifts of Sec. 3.1 and
 * Sec. 3.2): D^c = F^{c4} at an edge centre offset +1/2 along c;
 * B_c = (F_23, F_31, F_12)[c] at a face centre offset +1/2 along the two
 * axes other than c.  E_cov (= F_{c4}) and J^c share D's points; H (= F^{23},
 * F^{31}, F^{12}) shares B's points.  Nodes carry the mixed tensor.
 * ------------------------------------------------------------------ */

typedef struct {
    or_params p;
    int64_t ncap, n;       /* particle capacity and count (alive or dead) */
    double *x, *u;         /* SoA: x[3][ncap], u[4][ncap]                 */
    uint8_t *sp;           /* species, OR_DEAD when removed               */
    double *xold;          /* positions at the start of the step          */
    size_t gsize;          /* entries per ghosted field array             */
    double *D[3], *B[3], *E[3], *H[3], *J[3];
    double *rho_abs;       /* charge of particles removed at the horizon  */
    double *D0[3], *B0[3]; /* initial fields, targets of the inner relaxation */
    double *E0[3], *H0[3]; /* derived fields of the initial state            */
    int have_ref;
    double *node;          /* mixed tensor F^a_b at nodes, [node][16]     */
    int64_t gamma_clamps, n_removed_horizon, n_removed_outer, flags;
} or_sim;

static inline size_t gidx(const or_params *p, int i, int j, int k)
{
    return ((size_t)(k + 1) * (size_t)(p->ny + 3) + (size_t)(j + 1)) * (size_t)(p->nx + 3) +
           (size_t)(i + 1);
}

static inline size_t nidx(const or_params *p, int i, int j, int k)
{
    return ((size_t)k * (size_t)(p->ny + 1) + (size_t)j) * (size_t)(p->nx + 1) + (size_t)i;
}

static int ndim(const or_params *p, int axis)
{
    return axis == 0 ? p->nx : (axis == 1 ? p->ny : p->nz);
}

/* Half-offset pattern of each component: comp_off[kind][c][axis] with
 * kind 0 = E-type (D, E_cov, J) and kind 1 = B-type (B_cov, H). */
static int half_of(int kind, int c, int axis)
{
    if (kind == 0) return axis == c;
    return axis != c;
}

/* The inverse metric at a grid point, or Minkowski when r < r_exc.
 * reading: inside the excision radius the metric is never evaluated; the
 * flat metric stands in so derived quantities there stay finite. */
static void grid_metric(const or_params *p, double X, double Y, double Z,
                        double g[16], double gi[16])
{
    double x = X - p->center[0], y = Y - p->center[1], z = Z - p->center[2];
    double r = or_radius(p->a, x, y, z);
    if (r < p->r_exc) {
        for (int i = 0; i < 16; i++) {
            g[i] = 0.0;
            gi[i] = 0.0;
        }
        for (int i = 0; i < 4; i++) g[i * 5] = gi[i * 5] = ETA[i];
        return;
    }
    or_metric(p, x, y, z, g, gi, NULL);
}

static int excised(const or_params *p, double X, double Y, double Z)
{
    double x = X - p->center[0], y = Y - p->center[1], z = Z - p->center[2];
    return or_radius(p->a, x, y, z) < p->r_exc;
}

/* Pairs of the six independent components: s = {23, 31, 12}, t = {14, 24, 34}. */
static const int PS[3][2] = {{1, 2}, {2, 0}, {0, 1}};
static const int PT[3][2] = {{0, 3}, {1, 3}, {2, 3}};

/* Constitutive step (reading of "the same construction is used for the
 * contravariant and mixed field tensors", Sec. 3): from the evolved
 * covariant space pairs Fs_lo = (F_23, F_31, F_12) and contravariant time
 * pairs Ft_up = (F^14, F^24, F^34), recover Ft_lo = (F_14, F_24, F_34) and
 * Fs_up = (F^23, F^31, F^12) through F^{mn} = g^{ma} g^{nb} F_{ab}, written
 * as a 6x6 linear map M on the six pairs and solved for the unknown half.
 * Pinned: equals raising with the metric, F^{mn} = g^{ma} g^{nb} F_{ab},
 * at points around a spinning hole (random F), and its m=0 reduction
 * (E_cov = -D, H = B_cov). */
static void constitutive(const double gi[16], const double Fs_lo[3], const double Ft_up[3],
                         double Ft_lo[3], double Fs_up[3])
{
    int P[6][2];
    for (int i = 0; i < 3; i++) {
        P[i][0] = PS[i][0];
        P[i][1] = PS[i][1];
        P[i + 3][0] = PT[i][0];
        P[i + 3][1] = PT[i][1];
    }
    double M[6][6];
    for (int A = 0; A < 6; A++)
        for (int Bq = 0; Bq < 6; Bq++) {
            int mu = P[A][0], nu = P[A][1], al = P[Bq][0], be = P[Bq][1];
            M[A][Bq] = gi[mu * 4 + al] * gi[nu * 4 + be] - gi[mu * 4 + be] * gi[nu * 4 + al];
        }
    /* Solve M_tt Ft_lo = Ft_up - M_ts Fs_lo by elimination with pivoting. */
    double S[3][4];
    for (int i = 0; i < 3; i++) {
        double rhs = Ft_up[i];
        for (int j = 0; j < 3; j++) rhs -= M[i + 3][j] * Fs_lo[j];
        for (int j = 0; j < 3; j++) S[i][j] = M[i + 3][j + 3];
        S[i][3] = rhs;
    }
    for (int col = 0; col < 3; col++) {
        int piv = col;
        for (int i = col + 1; i < 3; i++)
            if (fabs(S[i][col]) > fabs(S[piv][col])) piv = i;
        if (piv != col)
            for (int j = 0; j < 4; j++) {
                double t = S[col][j];
                S[col][j] = S[piv][j];
                S[piv][j] = t;
            }
        for (int i = col + 1; i < 3; i++) {
            double fct = S[i][col] / S[col][col];
            for (int j = col; j < 4; j++) S[i][j] -= fct * S[col][j];
        }
    }
    for (int i = 2; i >= 0; i--) {
        double s = S[i][3];
        for (int j = i + 1; j < 3; j++) s -= S[i][j] * Ft_lo[j];
        Ft_lo[i] = s / S[i][i];
    }
    for (int i = 0; i < 3; i++) {
        double s = 0.0;
        for (int j = 0; j < 3; j++) s += M[i][j] * Fs_lo[j];
        for (int j = 0; j < 3; j++) s += M[i][j + 3] * Ft_lo[j];
        Fs_up[i] = s;
    }
}

/* Value of a staggered component (kind, c) averaged onto a point whose
 * half-offset pattern is pt_half[3] at integer index (i,j,k): along each
 * axis where the offsets agree the same index is used, otherwise the two
 * nearest points of the component (distance 1/2) are averaged.
 * reading: the paper does not say how off-point components are formed;
 * arithmetic means of the nearest neighbours are used.  Pinned through
 * the grid map below. */
static double avg_at(const or_params *p, const double *arr, int kind, int c,
                     const int pt_half[3], int i, int j, int k)
{
    int lo[3], hi[3];
    int idx[3] = {i, j, k};
    for (int ax = 0; ax < 3; ax++) {
        int ch = half_of(kind, c, ax);
        if (ch == pt_half[ax]) {
            lo[ax] = hi[ax] = idx[ax];
        } else if (ch == 1) { /* component at m+1/2, point at integer n: m = n-1, n */
            lo[ax] = idx[ax] - 1;
            hi[ax] = idx[ax];
        } else { /* component at integer m, point at n+1/2: m = n, n+1 */
            lo[ax] = idx[ax];
            hi[ax] = idx[ax] + 1;
        }
    }
    double s = 0.0;
    int cnt = 0;
    for (int kk = lo[2]; kk <= hi[2]; kk++)
        for (int jj = lo[1]; jj <= hi[1]; jj++)
            for (int ii = lo[0]; ii <= hi[0]; ii++) {
                s += arr[gidx(p, ii, jj, kk)];
                cnt++;
            }
    return s / (double)cnt;
}

/* Position (node coordinates) of the point (kind, c) at index (i,j,k). */
static void point_pos(int kind, int c, int i, int j, int k, double X[3])
{
    int idx[3] = {i, j, k};
    for (int ax = 0; ax < 3; ax++) X[ax] = (double)idx[ax] + (half_of(kind, c, ax) ? 0.5 : 0.0);
}

/* In-domain: integer axes in [0, n], half axes in [0, n-1]. */
static int in_domain(const or_params *p, int kind, int c, int i, int j, int k)
{
    int idx[3] = {i, j, k};
    for (int ax = 0; ax < 3; ax++) {
        int n = ndim(p, ax);
        if (half_of(kind, c, ax)) {
            if (idx[ax] < 0 || idx[ax] > n - 1) return 0;
        } else {
            if (idx[ax] < 0 || idx[ax] > n) return 0;
        }
    }
    return 1;
}

/* Updated: integer axes in [1, n-1] (the outermost node layers are held at
 * their initial values), half axes in [0, n-1], and not excised.
 * reading: the paper is silent on field boundaries. */
static int updated(const or_params *p, int kind, int c, int i, int j, int k)
{
    int idx[3] = {i, j, k};
    for (int ax = 0; ax < 3; ax++) {
        int n = ndim(p, ax);
        if (half_of(kind, c, ax)) {
            if (idx[ax] < 0 || idx[ax] > n - 1) return 0;
        } else {
            if (idx[ax] < 1 || idx[ax] > n - 1) return 0;
        }
    }
    double X[3];
    point_pos(kind, c, i, j, k, X);
    return !excised(p, X[0], X[1], X[2]);
}

/* Node values of the evolved pair: D^c averaged over the two E points next
 * to the node along c, B_c over the four B points around it. */
static void node_pair(const or_sim *s, int i, int j, int k, double vD[3], double vB[3])
{
    const or_params *p = &s->p;
    int ph[3] = {0, 0, 0};
    for (int q = 0; q < 3; q++) {
        vD[q] = avg_at(p, s->D[q], 0, q, ph, i, j, k);
        vB[q] = avg_at(p, s->B[q], 1, q, ph, i, j, k);
    }
}

/* Constitutive step on the grid (reading; the paper only says the same
 * construction serves the covariant, contravariant and mixed tensors).
 * Pointwise the map (D, B_cov) -> (-E_cov, H) is the symmetric matrix
 *   S = [[-M_tt^-1, M_tt^-1 M_ts], [M_st M_tt^-1, M_ss - M_st M_tt^-1 M_ts]]
 * obtained from constitutive() above, and S = I in flat space.  On the
 * staggered grid it is applied as
 *   (-E_cov, H) = (D, B_cov) + P^T (S - I) P (D, B_cov),
 * where P averages the six evolved components to the nodes (node_pair) and
 * P^T spreads a node value back with the same weights (1/2 to each of the
 * two E points, 1/4 to each of the four B points).  The map is symmetric,
 * so the field energy (D.D + B.B + sum over nodes of v.(S-I)v)/2 is an
 * invariant of the semi-discrete equations, and at m = 0 it is the Yee
 * identity.  Nodes that are excised or outside [0,n] contribute nothing.
 * Pinned: m = 0 reduction to Yee (cavity eigenmode recurrence); Wald's
 * vacuum solution in Kerr changes by a second-order truncation error per
 * cycle (the one-cycle change falls 8-fold when m, a and the grid double). */
static void compute_w(or_sim *s, double *w)
{
    const or_params *p = &s->p;
    for (int k = 0; k <= p->nz; k++)
        for (int j = 0; j <= p->ny; j++)
            for (int i = 0; i <= p->nx; i++) {
                double *o = w + 6 * nidx(p, i, j, k);
                if (excised(p, (double)i, (double)j, (double)k)) {
                    for (int q = 0; q < 6; q++) o[q] = 0.0;
                    continue;
                }
                double vD[3], vB[3], Ftl[3], Fsu[3], g[16], gi[16];
                node_pair(s, i, j, k, vD, vB);
                grid_metric(p, (double)i, (double)j, (double)k, g, gi);
                constitutive(gi, vB, vD, Ftl, Fsu);
                for (int q = 0; q < 3; q++) {
                    o[q] = -Ftl[q] - vD[q];
                    o[3 + q] = Fsu[q] - vB[q];
                }
            }
}

static int node_in(const or_params *p, int i, int j, int k)
{
    return i >= 0 && i <= p->nx && j >= 0 && j <= p->ny && k >= 0 && k <= p->nz;
}

/* E_cov = F_{c4} at every in-domain E point. */
static void compute_Ecov(or_sim *s)
{
    const or_params *p = &s->p;
    double *w = (double *)malloc(6 * (size_t)(p->nx + 1) * (p->ny + 1) * (p->nz + 1) * sizeof(double));
    compute_w(s, w);
    for (int c = 0; c < 3; c++)
        for (int k = 0; k <= p->nz; k++)
            for (int j = 0; j <= p->ny; j++)
                for (int i = 0; i <= p->nx; i++) {
                    if (!in_domain(p, 0, c, i, j, k)) continue;
                    double corr = 0.0;
                    for (int t = 0; t < 2; t++) {
                        int id[3] = {i, j, k};
                        id[c] += t;
                        if (node_in(p, id[0], id[1], id[2]))
                            corr += 0.5 * w[6 * nidx(p, id[0], id[1], id[2]) + c];
                    }
                    size_t g = gidx(p, i, j, k);
                    if (s->have_ref && !updated(p, 0, c, i, j, k))
                        s->E[c][g] = s->E0[c][g];
                    else
                        s->E[c][g] = -(s->D[c][g] + corr);
                }
    free(w);
}

/* H = F^{jk} at every in-domain B point. */
static void compute_H(or_sim *s)
{
    const or_params *p = &s->p;
    double *w = (double *)malloc(6 * (size_t)(p->nx + 1) * (p->ny + 1) * (p->nz + 1) * sizeof(double));
    compute_w(s, w);
    for (int c = 0; c < 3; c++) {
        int a1 = (c + 1) % 3, a2 = (c + 2) % 3;
        for (int k = 0; k <= p->nz; k++)
            for (int j = 0; j <= p->ny; j++)
                for (int i = 0; i <= p->nx; i++) {
                    if (!in_domain(p, 1, c, i, j, k)) continue;
                    double corr = 0.0;
                    for (int t1 = 0; t1 < 2; t1++)
                        for (int t2 = 0; t2 < 2; t2++) {
                            int id[3] = {i, j, k};
                            id[a1] += t1;
                            id[a2] += t2;
                            if (node_in(p, id[0], id[1], id[2]))
                                corr += 0.25 * w[6 * nidx(p, id[0], id[1], id[2]) + 3 + c];
                        }
                    size_t g = gidx(p, i, j, k);
                    if (s->have_ref && !updated(p, 1, c, i, j, k))
                        s->H[c][g] = s->H0[c][g];
                    else
                        s->H[c][g] = s->B[c][g] + corr;
                }
    }
    free(w);
}

/* Magnetic half-step (Sec. 3.1): for the covariant pair (al, be),
 *   F_{al be} -= [ (F_{be 4}(x + e_al) - F_{be 4}(x)) + (F_{4 al}(x + e_be) - F_{4 al}(x)) ] dx^4 / 2
 * with forward differences and F_{4 al} = -F_{al 4} = -E_cov[al]. */
static void b_half_step(or_sim *s)
{
    const or_params *p = &s->p;
    double h = 0.5 * p->c * p->dt;
    for (int c = 0; c < 3; c++) {
        int al = PS[c][0], be = PS[c][1];
        for (int k = 0; k <= p->nz; k++)
            for (int j = 0; j <= p->ny; j++)
                for (int i = 0; i <= p->nx; i++) {
                    if (!updated(p, 1, c, i, j, k)) continue;
                    int ia[3] = {i, j, k}, ib[3] = {i, j, k};
                    ia[al] += 1;
                    ib[be] += 1;
                    const double *Ebe = s->E[be], *Eal = s->E[al];
                    double d1 = Ebe[gidx(p, ia[0], ia[1], ia[2])] - Ebe[gidx(p, i, j, k)];
                    double d2 = -(Eal[gidx(p, ib[0], ib[1], ib[2])] - Eal[gidx(p, i, j, k)]);
                    s->B[c][gidx(p, i, j, k)] -= (d1 + d2) * h;
                }
    }
}

/* Electric full step (Sec. 3.2, continuous form of the update): with
 * sqrt(-g) = 1 both Christoffel terms vanish, leaving
 *   F^{c4} += dx^4 [ (4 pi / c) J^c - sum_k d_k F^{ck} ]
 * with backward differences of H = (F^23, F^31, F^12) at B points.
 * reading: the discrete form in the paper flips the sign of the current
 * term; the continuous form (which gives Ampere's law) is used. */
static void e_step(or_sim *s)
{
    const or_params *p = &s->p;
    double dx4 = p->c * p->dt;
    for (int c = 0; c < 3; c++) {
        for (int k = 0; k <= p->nz; k++)
            for (int j = 0; j <= p->ny; j++)
                for (int i = 0; i <= p->nx; i++) {
                    if (!updated(p, 0, c, i, j, k)) continue;
                    double div = 0.0;
                    for (int kk = 0; kk < 3; kk++) {
                        if (kk == c) continue;
                        /* F^{c kk} in terms of H: F^{ab} with (a,b) cyclic is H[the third axis]. */
                        int third = 3 - c - kk;
                        double sign = ((c + 1) % 3 == kk) ? 1.0 : -1.0; /* F^{c,c+1} = +H[c+2] */
                        int im[3] = {i, j, k};
                        im[kk] -= 1;
                        const double *Hh = s->H[third];
                        div += sign * (Hh[gidx(p, i, j, k)] - Hh[gidx(p, im[0], im[1], im[2])]);
                    }
                    size_t id = gidx(p, i, j, k);
                    s->D[c][id] += dx4 * ((4.0 * M_PI / p->c) * s->J[c][id] - div);
                }
    }
}

/* Time levels of the constitutive step (reading: the paper does not say at
 * which time level the index raising/lowering is taken).  The first
 * magnetic half-step needs E_cov at time n, which depends on B at time n
 * through the shift terms of g^{-1}; taking B at n-1/2 instead (an explicit
 * lag) advances those terms by forward Euler and grows without bound.
 * Instead E_cov^n is made consistent with B^n by a fixed number of
 * fixed-point passes of the half-step:
 *   B_(0) = B^{n-1/2};  E_(k) = C_E(D^n, B_(k));  B_(k+1) = B^{n-1/2} - (dx^4/2) curl E_(k),
 * k = 0..iters-1, so B^n = B_(iters) and the second half-step reuses
 * E_(iters-1).  The electric step is treated the same way around
 * D^{n+1/2} = (D^n + D^{n+1})/2 with H = C_H(B^{n+1/2}, D_(k)).  With one
 * pass this is the explicit lag; three passes give a time-centred,
 * non-growing update of the shift terms. */
static void copy3(double *dst[3], double *const src[3], size_t n)
{
    for (int c = 0; c < 3; c++) memcpy(dst[c], src[c], n * sizeof(double));
}

static void field_b_to_n(or_sim *s)
{
    int iters = s->p.field_iters > 0 ? s->p.field_iters : 1;
    double *B0[3];
    for (int c = 0; c < 3; c++) B0[c] = (double *)malloc(s->gsize * sizeof(double));
    copy3(B0, s->B, s->gsize);
    for (int it = 0; it < iters; it++) {
        compute_Ecov(s);
        copy3(s->B, B0, s->gsize);
        b_half_step(s);
    }
    for (int c = 0; c < 3; c++) free(B0[c]);
}

static void field_d_step(or_sim *s)
{
    int iters = s->p.field_iters > 0 ? s->p.field_iters : 1;
    double *D0[3];
    for (int c = 0; c < 3; c++) D0[c] = (double *)malloc(s->gsize * sizeof(double));
    copy3(D0, s->D, s->gsize);
    /* e_step with half the step gives D^{n+1/2}; the last pass takes the full step */
    double dt = s->p.dt;
    for (int it = 0; it < iters; it++) {
        compute_H(s);
        copy3(s->D, D0, s->gsize);
        if (it < iters - 1) {
            s->p.dt = 0.5 * dt;
            e_step(s);
            s->p.dt = dt;
        } else {
            e_step(s);
        }
    }
    for (int c = 0; c < 3; c++) free(D0[c]);
}

/* Whether the point lies in the relaxation layer (where Gauss's law is
 * deliberately not kept). */
static int relaxed(const or_params *p, int kind, int c, int i, int j, int k)
{
    if (!(p->r_damp > p->r_exc) || p->damp_max <= 0.0) return 0;
    double X[3];
    point_pos(kind, c, i, j, k, X);
    return or_radius(p->a, X[0] - p->center[0], X[1] - p->center[1], X[2] - p->center[2]) < p->r_damp;
}

/* Distance of a point from the nearest outer face of the grid. */
static double outer_distance(const or_params *p, const double X[3])
{
    double d = X[0];
    for (int ax = 0; ax < 3; ax++) {
        double lo = X[ax], hi = (double)ndim(p, ax) - X[ax];
        if (lo < d) d = lo;
        if (hi < d) d = hi;
    }
    return d;
}

/* Whether the point lies in the outer absorbing layer. */
static int in_outer_layer(const or_params *p, int kind, int c, int i, int j, int k)
{
    if (!(p->outer_layer > 0.0) || !(p->outer_damp > 0.0)) return 0;
    double X[3];
    point_pos(kind, c, i, j, k, X);
    return outer_distance(p, X) < p->outer_layer;
}

/* Relaxation inside the horizon (reading: the paper states no inner field
 * boundary).  Updated points with r_exc <= r < r_damp are pulled toward their
 * initial values by the fraction sigma = damp_max ((r_damp - r)/(r_damp - r_exc))^2
 * once per step, after the electric step.  The region is causally cut off
 * from the exterior, and without it the centred stencil grows near the
 * excision surface.  Pinned: one cycle with the layer equals the same cycle
 * without it followed by exactly this pull at exactly these points. */
static void relax_inner(or_sim *s)
{
    const or_params *p = &s->p;
    if (!(p->r_damp > p->r_exc) || p->damp_max <= 0.0) return;
    for (int kind = 0; kind < 2; kind++)
        for (int c = 0; c < 3; c++) {
            double *F = kind == 0 ? s->D[c] : s->B[c];
            const double *F0 = kind == 0 ? s->D0[c] : s->B0[c];
            for (int k = 0; k <= p->nz; k++)
                for (int j = 0; j <= p->ny; j++)
                    for (int i = 0; i <= p->nx; i++) {
                        if (!updated(p, kind, c, i, j, k)) continue;
                        double X[3];
                        point_pos(kind, c, i, j, k, X);
                        double r = or_radius(p->a, X[0] - p->center[0], X[1] - p->center[1],
                                             X[2] - p->center[2]);
                        if (r >= p->r_damp) continue;
                        double t = (p->r_damp - r) / (p->r_damp - p->r_exc);
                        double sg = p->damp_max * t * t;
                        size_t id = gidx(p, i, j, k);
                        F[id] -= sg * (F[id] - F0[id]);
                    }
        }
}

/* Outer absorbing layer (reading: the paper states no outer boundary
 * beyond the computational box; fields there are otherwise frozen, which
 * reflects outgoing waves).  Updated points closer than outer_layer to the
 * nearest outer face are pulled toward their initial values by
 * sigma = outer_damp ((outer_layer - d)/outer_layer)^2 once per step, after
 * the inner relaxation.  Pinned: a curl-free perturbation decays by exactly
 * (1 - sigma(d)) per step, and a vacuum pulse is absorbed instead of
 * reflected. */
static void relax_outer(or_sim *s)
{
    const or_params *p = &s->p;
    if (!(p->outer_layer > 0.0) || !(p->outer_damp > 0.0)) return;
    for (int kind = 0; kind < 2; kind++)
        for (int c = 0; c < 3; c++) {
            double *F = kind == 0 ? s->D[c] : s->B[c];
            const double *F0 = kind == 0 ? s->D0[c] : s->B0[c];
            for (int k = 0; k <= p->nz; k++)
                for (int j = 0; j <= p->ny; j++)
                    for (int i = 0; i <= p->nx; i++) {
                        if (!updated(p, kind, c, i, j, k)) continue;
                        double X[3];
                        point_pos(kind, c, i, j, k, X);
                        double d = outer_distance(p, X);
                        if (d >= p->outer_layer) continue;
                        double t = (p->outer_layer - d) / p->outer_layer;
                        double sg = p->outer_damp * t * t;
                        size_t id = gidx(p, i, j, k);
                        F[id] -= sg * (F[id] - F0[id]);
                    }
        }
}

/* Node tensor (Sec. 3.3, the field tensor components at the cell nodes):
 * average the staggered evolved pair to the node, complete it with the
 * constitutive step and lower the second index, F^a_b = F^{ag} g_{gb}.
 * reading: arithmetic means of the nearest neighbours.  Pinned: the
 * averaging (node_pair) and the constitutive step are those of the grid map
 * (Wald convergence, pointwise raising); the lowering uses the pinned
 * metric. */
static void compute_nodes(or_sim *s)
{
    const or_params *p = &s->p;
    for (int k = 0; k <= p->nz; k++)
        for (int j = 0; j <= p->ny; j++)
            for (int i = 0; i <= p->nx; i++) {
                double Fs[3], Ft[3], Ftl[3], Fsu[3], g[16], gi[16];
                node_pair(s, i, j, k, Ft, Fs);
                grid_metric(p, (double)i, (double)j, (double)k, g, gi);
                constitutive(gi, Fs, Ft, Ftl, Fsu);
                double F[4][4];
                memset(F, 0, sizeof(F));
                for (int q = 0; q < 3; q++) {
                    F[PS[q][0]][PS[q][1]] = Fsu[q];
                    F[PS[q][1]][PS[q][0]] = -Fsu[q];
                    F[PT[q][0]][PT[q][1]] = Ft[q];
                    F[PT[q][1]][PT[q][0]] = -Ft[q];
                }
                double *out = s->node + 16 * nidx(p, i, j, k);
                for (int al = 0; al < 4; al++)
                    for (int be = 0; be < 4; be++) {
                        double v = 0.0;
                        for (int ga = 0; ga < 4; ga++) v += F[al][ga] * g[ga * 4 + be];
                        out[al * 4 + be] = v;
                    }
            }
}

/* ------------------------------------------------------------------ */
/* Gather (Sec. 3.3): cloud-in-cell weights from sub-volumes
 * VOLUME = int sqrt(-det g) dx^1 dx^2 dx^3.  Since det g = -1 exactly for
 * this metric (pinned), the sub-volumes are Euclidean and the weights are
 * the trilinear ones.  reading: the cell is floor(X) clamped to the grid
 * and the fractional offset is not clamped, so a stage position just
 * outside the grid extrapolates linearly.  Pinned: weights sum to one and
 * a linear field is reproduced exactly. */
/* Spatial volume density sqrt(det g_ij), i, j = 1..3, at a hole-relative
 * point: the determinant of the spatial block of the metric, written out;
 * 1 inside the excision radius (those points are flat, as in the field
 * solve).  Used by gather reading B only. */
double or_spatial_density(const or_params *p, double x, double y, double z)
{
    if (p->m == 0.0) return 1.0;
    double g[16], r;
    or_metric(p, x, y, z, g, NULL, &r);
    if (r < p->r_exc) return 1.0;
    double det = g[0] * (g[5] * g[10] - g[6] * g[9]) - g[1] * (g[4] * g[10] - g[6] * g[8]) +
                 g[2] * (g[4] * g[9] - g[5] * g[8]);
    return sqrt(det);
}

/* Cloud-in-cell weights of the 8 nodes of cell c for a particle at X.
 * gather_weights 0: the sub-volume opposite each node with the 4-metric
 * density sqrt(-det g) = 1, i.e. the trilinear weights.  gather_weights 1
 * (reading B, an ablation): the sub-volume weighted by the spatial density
 * sqrt(det g_ij) at its centre (midpoint rule), normalised by the sum.
 * Pinned: reading B equals trilinear at m = 0, sums to one, keeps a
 * constant field, is mirror symmetric where the density is, and its
 * sub-volumes approach a high-order quadrature at second order. */
void or_gather_weights(const or_params *p, const int c[3], const double X[3], double W[8])
{
    double sum = 0.0;
    for (int dk = 0; dk < 2; dk++)
        for (int dj = 0; dj < 2; dj++)
            for (int di = 0; di < 2; di++) {
                /* the sub-volume opposite the node spans [X, c+1] on axes
                 * where the node is at c and [c, X] where it is at c+1 */
                int d[3] = {di, dj, dk};
                double w[3], mid[3];
                for (int ax = 0; ax < 3; ax++) {
                    w[ax] = X[ax] - (double)c[ax];
                    mid[ax] = d[ax] ? 0.5 * ((double)c[ax] + X[ax]) : 0.5 * (X[ax] + (double)c[ax] + 1.0);
                }
                double V = (di ? w[0] : 1.0 - w[0]) * (dj ? w[1] : 1.0 - w[1]) * (dk ? w[2] : 1.0 - w[2]);
                if (p->gather_weights == 1)
                    V *= or_spatial_density(p, mid[0] - p->center[0], mid[1] - p->center[1],
                                            mid[2] - p->center[2]);
                W[di + 2 * dj + 4 * dk] = V;
                sum += V;
            }
    if (p->gather_weights == 1)
        for (int n = 0; n < 8; n++) W[n] /= sum;
}

void or_gather(const or_params *p, const double *node, const double X[3], double Fo[16])
{
    int c[3];
    for (int ax = 0; ax < 3; ax++) {
        int n = ndim(p, ax);
        int ci = (int)floor(X[ax]);
        if (ci < 0) ci = 0;
        if (ci > n - 1) ci = n - 1;
        c[ax] = ci;
    }
    double W[8];
    or_gather_weights(p, c, X, W);
    for (int q = 0; q < 16; q++) Fo[q] = 0.0;
    for (int dk = 0; dk < 2; dk++)
        for (int dj = 0; dj < 2; dj++)
            for (int di = 0; di < 2; di++) {
                const double *src = node + 16 * nidx(p, c[0] + di, c[1] + dj, c[2] + dk);
                for (int q = 0; q < 16; q++) Fo[q] += W[di + 2 * dj + 4 * dk] * src[q];
            }
}

/* ------------------------------------------------------------------ */
/* Equation of motion (Sec. 3.3):
 *   du^a/dtau = (q/m) F^a_b u^b - Gamma^a_{mn} u^m u^n.
 * reading: as printed, with no 1/c on the Lorentz term.  Fpre, when not
 * NULL, is the field tensor to use instead of the gather at X (the
 * per-step gather ablation); the Christoffel symbols are always taken at X,
 * as the paper states for the push. */
static void accel(const or_params *p, const double *node, const double *Fpre, double qm,
                  const double X[3], const double u[4], double A[4])
{
    double G[64];
    or_christoffel(p, X[0] - p->center[0], X[1] - p->center[1], X[2] - p->center[2], G);
    double F[16];
    if (Fpre)
        for (int q = 0; q < 16; q++) F[q] = Fpre[q];
    else if (node && qm != 0.0)
        or_gather(p, node, X, F);
    else
        for (int q = 0; q < 16; q++) F[q] = 0.0;
    for (int a = 0; a < 4; a++) {
        double lor = 0.0;
        for (int b = 0; b < 4; b++) lor += F[a * 4 + b] * u[b];
        double gam = 0.0;
        for (int mu = 0; mu < 4; mu++)
            for (int nu = 0; nu < 4; nu++) gam += G[a * 16 + mu * 4 + nu] * u[mu] * u[nu];
        A[a] = qm * lor - gam;
    }
}

/* Time-dilation factor for a stage (eq. for gamma_i in Sec. 3.3):
 * mode 0 takes the printed estimate 1/2 [u4/c + sqrt((u4/c)^2 + 4 a4 dt/(2c))],
 * a negative discriminant clamped to zero and counted; mode 1 takes
 * u4/c, the limit of that estimate for dt -> 0. */
static double stage_gamma(const or_params *p, double u4, double a4, int64_t *clamps)
{
    double c = p->c;
    if (p->gamma_mode == 1) return u4 / c;
    double disc = (u4 / c) * (u4 / c) + 4.0 * a4 * (p->dt / (2.0 * c));
    if (disc < 0.0) {
        disc = 0.0;
        if (clamps) (*clamps)++;
    }
    return 0.5 * (u4 / c + sqrt(disc));
}

/* Field tensor for the per-step gather ablation (gather_mode 1): the
 * gather at the step's start position, used unchanged by all four stages.
 * Returns NULL (gather at every stage) in the default mode or when the
 * particle feels no field. */
static const double *step_fields(const or_params *p, const double *node, double qm, const double X[3],
                                 double F[16])
{
    if (p->gather_mode != 1 || !node || qm == 0.0) return NULL;
    or_gather(p, node, X, F);
    return F;
}

/* One RK4 step in coordinate time of Y = (x^1..3, u^1..4).
 * reading of the printed steps (whose final weights sum to 5/6 and whose
 * half-velocity averaging fails constant-acceleration kinematics): stage k
 * evaluates A_k and gamma_k at Y_k and the slope K_k = (u_k, A_k)/gamma_k,
 * so dt*K_k = (u_k, A_k) dtau_k with dtau_k = dt/gamma_k; then
 * Y_2 = Y_n + dt/2 K_1, Y_3 = Y_n + dt/2 K_2, Y_4 = Y_n + dt K_3,
 * Y_{n+1} = Y_n + dt/6 (K_1 + 2 K_2 + 2 K_3 + K_4).  Fields and
 * Christoffel symbols are evaluated at every stage position (fields at
 * x_n only with gather_mode 1).
 * Pinned: m=0 gyration equals the RK4 stability polynomial, E x B drift,
 * circular and inclined Kerr orbits, convergence order; with gather_mode 1,
 * the RK4 polynomial of the field frozen at x_n in a linear field. */
static void rk4_step(const or_params *p, const double *node, double qm,
                     double X[3], double u[4], int64_t *clamps)
{
    double dt = p->dt;
    double Y0[7], Yk[7], K[4][7];
    for (int i = 0; i < 3; i++) Y0[i] = X[i];
    for (int i = 0; i < 4; i++) Y0[3 + i] = u[i];
    for (int i = 0; i < 7; i++) Yk[i] = Y0[i];
    double F0[16];
    const double *Fpre = step_fields(p, node, qm, X, F0);
    static const double fac[3] = {0.5, 0.5, 1.0};
    for (int st = 0; st < 4; st++) {
        double A[4];
        accel(p, node, Fpre, qm, &Yk[0], &Yk[3], A);
        double gam = stage_gamma(p, Yk[6], A[3], clamps);
        for (int i = 0; i < 3; i++) K[st][i] = Yk[3 + i] / gam;
        for (int i = 0; i < 4; i++) K[st][3 + i] = A[i] / gam;
        if (st < 3)
            for (int i = 0; i < 7; i++) Yk[i] = Y0[i] + fac[st] * dt * K[st][i];
    }
    for (int i = 0; i < 7; i++)
        Yk[i] = Y0[i] + (dt / 6.0) * (K[0][i] + 2.0 * K[1][i] + 2.0 * K[2][i] + K[3][i]);
    for (int i = 0; i < 3; i++) X[i] = Yk[i];
    for (int i = 0; i < 4; i++) u[i] = Yk[3 + i];
}

/* The four steps exactly as printed in Sec. 3.3 (rk_mode 1, an ablation of
 * the reading above), with the two final sums read as increments added to
 * x_n and u_n.  Step k (k = 1..4) takes the averaged velocity
 * ut_k = (u_n + u_k)/2 (ut_1 = u_n) and the position
 * x_k = x_n + ut_k dtau_{k-1} (x_1 = x_n), evaluates a_k = a(x_k, ut_k) and
 * gamma_k = f(ut_k^4, a_k^4), with dtau_1 = dt/(2 gamma_1),
 * dtau_2,3 = dt/gamma_2,3, dtau_4 = dt/(2 gamma_4), and
 * u_{k+1} = u_n + a_k dtau_k; then
 *   x_{n+1} = x_n + (ut_1 dtau_1 + 2 (ut_2 dtau_2 + ut_3 dtau_3) + ut_4 dtau_4)/6,
 *   u_{n+1} = u_n + (a_1 dtau_1 + 2 (a_2 dtau_2 + a_3 dtau_3) + a_4 dtau_4)/6.
 * Pinned: for du/dtau = Omega u with constant gamma (m = 0, uniform B) the
 * step is the polynomial I + 5M/6 + 7M^2/24 + M^3/16 + M^4/192 of
 * M = Omega dt/gamma, and a free particle moves 5/6 of v dt. */
static void rk4_literal_step(const or_params *p, const double *node, double qm,
                             double X[3], double u[4], int64_t *clamps)
{
    double dt = p->dt;
    double x0[3], u0[4], xk[3], ut[4], uk[4];
    double sx[3] = {0.0, 0.0, 0.0}, su[4] = {0.0, 0.0, 0.0, 0.0};
    for (int i = 0; i < 3; i++) x0[i] = xk[i] = X[i];
    for (int i = 0; i < 4; i++) u0[i] = ut[i] = uk[i] = u[i];
    double F0[16];
    const double *Fpre = step_fields(p, node, qm, X, F0);
    double dtau_prev = 0.0;
    for (int st = 0; st < 4; st++) {
        if (st > 0) {
            for (int i = 0; i < 4; i++) ut[i] = 0.5 * (u0[i] + uk[i]);
            for (int i = 0; i < 3; i++) xk[i] = x0[i] + ut[i] * dtau_prev;
        }
        double A[4];
        accel(p, node, Fpre, qm, xk, ut, A);
        double gam = stage_gamma(p, ut[3], A[3], clamps);
        double dtau = (st == 0 || st == 3) ? dt / (2.0 * gam) : dt / gam;
        double w = (st == 0 || st == 3) ? 1.0 : 2.0;
        for (int i = 0; i < 3; i++) sx[i] += w * ut[i] * dtau;
        for (int i = 0; i < 4; i++) su[i] += w * A[i] * dtau;
        for (int i = 0; i < 4; i++) uk[i] = u0[i] + A[i] * dtau;
        dtau_prev = dtau;
    }
    for (int i = 0; i < 3; i++) X[i] = x0[i] + sx[i] / 6.0;
    for (int i = 0; i < 4; i++) u[i] = u0[i] + su[i] / 6.0;
}

/* The push of one particle in the configured reading. */
static void push_step(const or_params *p, const double *node, double qm, double X[3], double u[4],
                      int64_t *clamps)
{
    if (p->rk_mode == 1)
        rk4_literal_step(p, node, qm, X, u, clamps);
    else
        rk4_step(p, node, qm, X, u, clamps);
}

/* ------------------------------------------------------------------ */
/* Current deposition (Sec. 4).
 * reading: the chord x_n -> x_{n+1} is split per axis at the relay point
 *   x_r = min(min(i1,i2)+1, max(max(i1,i2), (x1+x2)/2))
 * into two segments each inside one cell; a segment carries the flux
 * FLUX^K = q dx^K / dt through the K-face (J = rho u with the proper
 * density, so no extra gamma).  Transverse weights over the (I,J) face:
 *  - curved: AREA of each sub-rectangle by the midpoint rule with density
 *    sqrt(g_II g_JJ - g_IJ^2) at the sub-rectangle centre in the plane of
 *    the segment midpoint, normalised by their sum (FACE_AREA); node (i,j)
 *    takes the sub-rectangle opposite to it;
 *  - flat: the bilinear weights at the segment midpoint;
 * both plus the exact segment-average term +-dI dJ/12 (+ on (i,j) and
 * (i+1,j+1)).  Pinned: discrete continuity in flat mode and at m=0, flux
 * sum, curved == flat at m=0, and each curved weight against a 5x5
 * Gauss-Legendre integral of the density over its sub-rectangle (within the
 * midpoint rule's O(h^2) error; the density at a wrong point fails). */
static double area_density(const or_params *p, int I, int Jx, const double X[3])
{
    double x = X[0] - p->center[0], y = X[1] - p->center[1], z = X[2] - p->center[2];
    double r = or_radius(p->a, x, y, z);
    if (r < p->r_exc) return 1.0;
    double g[16];
    or_metric(p, x, y, z, g, NULL, NULL);
    double v = g[I * 4 + I] * g[Jx * 4 + Jx] - g[I * 4 + Jx] * g[Jx * 4 + I];
    return sqrt(v);
}

static void deposit_segment(or_sim *s, const double A[3], const double Bp[3],
                            const int cell[3], double Q)
{
    const or_params *p = &s->p;
    double d[3], mid[3];
    for (int ax = 0; ax < 3; ax++) {
        d[ax] = Bp[ax] - A[ax];
        mid[ax] = 0.5 * (A[ax] + Bp[ax]);
    }
    for (int K = 0; K < 3; K++) {
        int I = (K + 1) % 3, Jx = (K + 2) % 3;
        double flux = Q * d[K] / p->dt;
        if (flux == 0.0) continue;
        double t = d[I] * d[Jx] / 12.0;
        double w[2][2];
        double lo_I = (double)cell[I], lo_J = (double)cell[Jx];
        if (p->deposit_mode == 1) {
            double xi = mid[I] - lo_I, eta = mid[Jx] - lo_J;
            w[0][0] = (1.0 - xi) * (1.0 - eta);
            w[1][0] = xi * (1.0 - eta);
            w[0][1] = (1.0 - xi) * eta;
            w[1][1] = xi * eta;
        } else {
            double area[2][2], tot = 0.0;
            for (int bj = 0; bj < 2; bj++)
                for (int bi = 0; bi < 2; bi++) {
                    /* node (lo+bi, lo+bj) takes the opposite sub-rectangle */
                    double i0 = bi ? lo_I : mid[I], i1 = bi ? mid[I] : lo_I + 1.0;
                    double j0 = bj ? lo_J : mid[Jx], j1 = bj ? mid[Jx] : lo_J + 1.0;
                    double P[3];
                    P[K] = mid[K];
                    P[I] = 0.5 * (i0 + i1);
                    P[Jx] = 0.5 * (j0 + j1);
                    area[bi][bj] = area_density(p, I, Jx, P) * (i1 - i0) * (j1 - j0);
                }
            for (int bj = 0; bj < 2; bj++)
                for (int bi = 0; bi < 2; bi++) tot += area[bi][bj];
            for (int bj = 0; bj < 2; bj++)
                for (int bi = 0; bi < 2; bi++) w[bi][bj] = area[bi][bj] / tot;
        }
        w[0][0] += t;
        w[1][1] += t;
        w[1][0] -= t;
        w[0][1] -= t;
        for (int bj = 0; bj < 2; bj++)
            for (int bi = 0; bi < 2; bi++) {
                int id[3];
                id[K] = cell[K];
                id[I] = cell[I] + bi;
                id[Jx] = cell[Jx] + bj;
                s->J[K][gidx(p, id[0], id[1], id[2])] += flux * w[bi][bj];
            }
    }
}

static void deposit_particle(or_sim *s, const double x1[3], const double x2[3], double Q)
{
    double xr[3];
    int c1[3], c2[3];
    for (int ax = 0; ax < 3; ax++) {
        int i1 = (int)floor(x1[ax]), i2 = (int)floor(x2[ax]);
        double lo = (double)((i1 < i2 ? i1 : i2) + 1);
        double hi = (double)(i1 > i2 ? i1 : i2);
        double mid = 0.5 * (x1[ax] + x2[ax]);
        double v = mid > hi ? mid : hi;
        xr[ax] = v < lo ? v : lo;
        c1[ax] = i1;
        c2[ax] = i2;
    }
    for (int ax = 0; ax < 3; ax++) {
        int n = ndim(&s->p, ax);
        if (c1[ax] < -1 || c1[ax] > n || c2[ax] < -1 || c2[ax] > n ||
            fabs(x2[ax] - x1[ax]) >= 1.0) {
            s->flags |= 1; /* move longer than one cell or outside the ghost layer */
            return;
        }
    }
    deposit_segment(s, x1, xr, c1, Q);
    deposit_segment(s, xr, x2, c2, Q);
}

/* Trilinear charge of one particle onto nodes of a ghosted array. */
static void deposit_charge(const or_params *p, double *rho, const double X[3], double Q)
{
    int c[3];
    double w[3];
    for (int ax = 0; ax < 3; ax++) {
        c[ax] = (int)floor(X[ax]);
        w[ax] = X[ax] - (double)c[ax];
    }
    for (int dk = 0; dk < 2; dk++)
        for (int dj = 0; dj < 2; dj++)
            for (int di = 0; di < 2; di++) {
                double W = (di ? w[0] : 1.0 - w[0]) * (dj ? w[1] : 1.0 - w[1]) *
                           (dk ? w[2] : 1.0 - w[2]);
                rho[gidx(p, c[0] + di, c[1] + dj, c[2] + dk)] += Q * W;
            }
}

/* ------------------------------------------------------------------ */
/* Simulation object.                                                  */
/* ------------------------------------------------------------------ */

or_sim *or_sim_new(const or_params *p, int64_t ncap)
{
    or_sim *s = (or_sim *)calloc(1, sizeof(or_sim));
    if (!s) return NULL;
    s->p = *p;
    s->ncap = ncap;
    s->n = 0;
    size_t nc = (size_t)(ncap > 0 ? ncap : 1);
    s->x = (double *)calloc(3 * nc, sizeof(double));
    s->xold = (double *)calloc(3 * nc, sizeof(double));
    s->u = (double *)calloc(4 * nc, sizeof(double));
    s->sp = (uint8_t *)calloc(nc, 1);
    s->gsize = (size_t)(p->nx + 3) * (size_t)(p->ny + 3) * (size_t)(p->nz + 3);
    for (int c = 0; c < 3; c++) {
        s->D[c] = (double *)calloc(s->gsize, sizeof(double));
        s->B[c] = (double *)calloc(s->gsize, sizeof(double));
        s->E[c] = (double *)calloc(s->gsize, sizeof(double));
        s->H[c] = (double *)calloc(s->gsize, sizeof(double));
        s->J[c] = (double *)calloc(s->gsize, sizeof(double));
        s->D0[c] = (double *)calloc(s->gsize, sizeof(double));
        s->B0[c] = (double *)calloc(s->gsize, sizeof(double));
        s->E0[c] = (double *)calloc(s->gsize, sizeof(double));
        s->H0[c] = (double *)calloc(s->gsize, sizeof(double));
    }
    s->rho_abs = (double *)calloc(s->gsize, sizeof(double));
    s->node = (double *)calloc(16 * (size_t)(p->nx + 1) * (p->ny + 1) * (p->nz + 1), sizeof(double));
    return s;
}

void or_sim_free(or_sim *s)
{
    if (!s) return;
    free(s->x);
    free(s->xold);
    free(s->u);
    free(s->sp);
    for (int c = 0; c < 3; c++) {
        free(s->D[c]);
        free(s->B[c]);
        free(s->E[c]);
        free(s->H[c]);
        free(s->J[c]);
        free(s->D0[c]);
        free(s->B0[c]);
        free(s->E0[c]);
        free(s->H0[c]);
    }
    free(s->rho_abs);
    free(s->node);
    free(s);
}

size_t or_sim_gsize(const or_sim *s) { return s->gsize; }


/* Reference (initial) state.  Points that are not updated (outermost node
 * layers, ghosts, excised points) hold their evolved values and also their
 * derived E_cov and H at the values of the initial state; with that, the
 * energy of a perturbation of the initial state has no flux through the
 * frozen points (reading: the paper states no field boundary). */
static void set_reference(or_sim *s)
{
    for (int c = 0; c < 3; c++) {
        memcpy(s->D0[c], s->D[c], s->gsize * sizeof(double));
        memcpy(s->B0[c], s->B[c], s->gsize * sizeof(double));
    }
    s->have_ref = 0;
    compute_Ecov(s);
    compute_H(s);
    for (int c = 0; c < 3; c++) {
        memcpy(s->E0[c], s->E[c], s->gsize * sizeof(double));
        memcpy(s->H0[c], s->H[c], s->gsize * sizeof(double));
    }
    s->have_ref = 1;
}

/* Initial fields.  covariant = 0: uniform contravariant F^{23}, F^{31},
 * F^{12} = B0 with F^{j4} = 0 (the application section takes the
 * contravariant z component uniform); the evolved covariant pairs are the
 * full lowering F_ab = g_am g_bn F^{mn} at every B point.  covariant = 1:
 * uniform covariant F_23, F_31, F_12 = B0 with F_{j4} = 0, which for a = 0
 * and B0 along z is Wald's static vacuum solution A = (B0/2)(x dy - y dx);
 * D = F^{j4} is the full raising at every E point.  Flat metric inside r_exc. */
void or_sim_init_fields2(or_sim *s, const double B0[3], int covariant)
{
    const or_params *p = &s->p;
    double F[4][4];
    memset(F, 0, sizeof(F));
    for (int q = 0; q < 3; q++) {
        F[PS[q][0]][PS[q][1]] = B0[q];
        F[PS[q][1]][PS[q][0]] = -B0[q];
    }
    for (int c = 0; c < 3; c++) {
        memset(s->D[c], 0, s->gsize * sizeof(double));
        memset(s->E[c], 0, s->gsize * sizeof(double));
        memset(s->H[c], 0, s->gsize * sizeof(double));
        memset(s->J[c], 0, s->gsize * sizeof(double));
    }
    memset(s->rho_abs, 0, s->gsize * sizeof(double));
    for (int kind = 0; kind < 2; kind++)
        for (int c = 0; c < 3; c++) {
            int al = kind == 1 ? PS[c][0] : PT[c][0];
            int be = kind == 1 ? PS[c][1] : PT[c][1];
            for (int k = -1; k <= p->nz + 1; k++)
                for (int j = -1; j <= p->ny + 1; j++)
                    for (int i = -1; i <= p->nx + 1; i++) {
                        double X[3], g[16], gi[16];
                        point_pos(kind, c, i, j, k, X);
                        grid_metric(p, X[0], X[1], X[2], g, gi);
                        const double *T = covariant ? gi : g;
                        double v = 0.0;
                        for (int mu = 0; mu < 4; mu++)
                            for (int nu = 0; nu < 4; nu++)
                                v += T[al * 4 + mu] * T[be * 4 + nu] * F[mu][nu];
                        if (kind == 1)
                            s->B[c][gidx(p, i, j, k)] = covariant ? B0[c] : v;
                        else
                            s->D[c][gidx(p, i, j, k)] = covariant ? v : 0.0;
                    }
        }
    set_reference(s);
}

void or_sim_init_fields(or_sim *s, const double B0[3]) { or_sim_init_fields2(s, B0, 0); }

/* Take the current fields as the reference state: the values the frozen
 * points hold and the relaxation layers pull toward (test hook, used to
 * start from a stationary solution other than the paper's initial field). */
void or_sim_make_reference(or_sim *s) { set_reference(s); }

/* Test hook: the constitutive step of the grid at one point (node
 * coordinates X, Y, Z; the flat metric inside r_exc), from (F_23, F_31,
 * F_12) and (F^14, F^24, F^34) to (F_14, F_24, F_34) and (F^23, F^31, F^12). */
void or_constitutive_point(const or_params *p, double X, double Y, double Z, const double Fs_lo[3],
                           const double Ft_up[3], double Ft_lo[3], double Fs_up[3])
{
    double g[16], gi[16];
    grid_metric(p, X, Y, Z, g, gi);
    constitutive(gi, Fs_lo, Ft_up, Ft_lo, Fs_up);
}

void or_sim_set_fields(or_sim *s, const double *D, const double *B)
{
    for (int c = 0; c < 3; c++) {
        memcpy(s->D[c], D + c * s->gsize, s->gsize * sizeof(double));
        memcpy(s->B[c], B + c * s->gsize, s->gsize * sizeof(double));
    }
}



/* which: 0 D, 1 B_cov, 2 E_cov, 3 H, 4 J, 5 rho_abs (one component) */
void or_sim_get_fields(const or_sim *s, int which, double *out)
{
    if (which == 5) {
        memcpy(out, s->rho_abs, s->gsize * sizeof(double));
        return;
    }
    for (int c = 0; c < 3; c++) {
        const double *src = which == 0 ? s->D[c]
                          : which == 1 ? s->B[c]
                          : which == 2 ? s->E[c]
                          : which == 3 ? s->H[c]
                                       : s->J[c];
        memcpy(out + c * s->gsize, src, s->gsize * sizeof(double));
    }
}

size_t or_sim_node_count(const or_sim *s)
{
    return (size_t)(s->p.nx + 1) * (s->p.ny + 1) * (s->p.nz + 1);
}

void or_sim_compute_nodes(or_sim *s) { compute_nodes(s); }
void or_sim_compute_derived(or_sim *s)
{
    compute_Ecov(s);
    compute_H(s);
}

void or_sim_get_nodes(const or_sim *s, double *out)
{
    memcpy(out, s->node, 16 * or_sim_node_count(s) * sizeof(double));
}

void or_sim_set_nodes(or_sim *s, const double *in)
{
    memcpy(s->node, in, 16 * or_sim_node_count(s) * sizeof(double));
}

/* Set particles verbatim: x[3][n], u[4][n] contravariant, sp[n]. */
int or_sim_set_particles(or_sim *s, int64_t n, const double *x, const double *u, const uint8_t *sp)
{
    if (n > s->ncap) return -1;
    s->n = n;
    for (int64_t i = 0; i < n; i++) {
        for (int ax = 0; ax < 3; ax++) s->x[ax * s->ncap + i] = x[ax * n + i];
        for (int c = 0; c < 4; c++) s->u[c * s->ncap + i] = u[c * n + i];
        s->sp[i] = sp[i];
    }
    return 0;
}

void or_sim_get_particles(const or_sim *s, double *x, double *u, uint8_t *sp)
{
    int64_t n = s->n;
    for (int64_t i = 0; i < n; i++) {
        for (int ax = 0; ax < 3; ax++) x[ax * n + i] = s->x[ax * s->ncap + i];
        for (int c = 0; c < 4; c++) u[c * n + i] = s->u[c * s->ncap + i];
        sp[i] = s->sp[i];
    }
}

int64_t or_sim_count(const or_sim *s) { return s->n; }

/* Future-directed four-velocity from the spatial covariant components
 * u_1..3 and the mass shell g_{mn} u^m u^n = -c^2 (Sec. 2.1, time
 * dilation relation): g^{44} u_4^2 + 2 (g^{4i} u_i) u_4 + g^{ij} u_i u_j + c^2 = 0,
 * root with u^4 = g^{4b} u_b > 0, then u^a = g^{ab} u_b.
 * reading: the particle input carries covariant spatial components so
 * that the shell always has a future root (dx^4 is timelike everywhere
 * outside r = 0).  Pinned: shell residual, covariant components returned. */
void or_mass_shell(const or_params *p, const double X[3], const double ucov[3], double uout[4])
{
    double g[16], gi[16];
    or_metric(p, X[0] - p->center[0], X[1] - p->center[1], X[2] - p->center[2], g, gi, NULL);
    double c = p->c;
    double A = gi[15];
    double B = 0.0, C = c * c;
    for (int i = 0; i < 3; i++) B += gi[12 + i] * ucov[i];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) C += gi[i * 4 + j] * ucov[i] * ucov[j];
    double disc = B * B - A * C;
    if (disc < 0.0) disc = 0.0;
    double sq = sqrt(disc);
    /* u^4 = A u_4 + B = +sq */
    double u4low = (B <= 0.0) ? (sq - B) / A : -C / (sq + B);
    double ul[4] = {ucov[0], ucov[1], ucov[2], u4low};
    for (int a = 0; a < 4; a++) {
        double v = 0.0;
        for (int b = 0; b < 4; b++) v += gi[a * 4 + b] * ul[b];
        uout[a] = v;
    }
}

static int outside_grid(const or_params *p, const double X[3])
{
    for (int ax = 0; ax < 3; ax++) {
        double n = (double)ndim(p, ax);
        if (!(X[ax] >= 0.0 && X[ax] < n)) return 1;
    }
    return 0;
}

/* Load particles of one species from positions and covariant spatial
 * four-velocities; drops particles inside r_rm or outside the grid
 * (reading: the paper states no particle boundary).  Returns the number kept. */
int64_t or_sim_load(or_sim *s, int species, int64_t n, const double *x, const double *ucov)
{
    const or_params *p = &s->p;
    int64_t kept = 0;
    for (int64_t i = 0; i < n; i++) {
        double X[3] = {x[i], x[n + i], x[2 * n + i]};
        double uc[3] = {ucov[i], ucov[n + i], ucov[2 * n + i]};
        if (outside_grid(p, X)) continue;
        double r = or_radius(p->a, X[0] - p->center[0], X[1] - p->center[1], X[2] - p->center[2]);
        if (r < p->r_rm) continue;
        if (s->n >= s->ncap) return -1;
        double U[4];
        or_mass_shell(p, X, uc, U);
        int64_t j = s->n++;
        for (int ax = 0; ax < 3; ax++) s->x[ax * s->ncap + j] = X[ax];
        for (int c = 0; c < 4; c++) s->u[c * s->ncap + j] = U[c];
        s->sp[j] = (uint8_t)species;
        kept++;
    }
    return kept;
}

/* Push the live particles through nsteps RK4 steps with the node tensor
 * frozen (node may be NULL: no electromagnetic force).  Test-particle
 * mode; no deposition or removal. */
void or_sim_push_only(or_sim *s, int nsteps, int use_nodes)
{
    const or_params *p = &s->p;
    for (int st = 0; st < nsteps; st++)
        for (int64_t i = 0; i < s->n; i++) {
            if (s->sp[i] == OR_DEAD) continue;
            int sp = s->sp[i];
            double qm = p->mass[sp] != 0.0 ? p->charge[sp] / p->mass[sp] : 0.0;
            double X[3], U[4];
            for (int ax = 0; ax < 3; ax++) X[ax] = s->x[ax * s->ncap + i];
            for (int c = 0; c < 4; c++) U[c] = s->u[c * s->ncap + i];
            push_step(p, use_nodes ? s->node : NULL, qm, X, U, &s->gamma_clamps);
            for (int ax = 0; ax < 3; ax++) s->x[ax * s->ncap + i] = X[ax];
            for (int c = 0; c < 4; c++) s->u[c * s->ncap + i] = U[c];
        }
}

/* The first half of a cycle: magnetic half-step to B^n with the
 * self-consistent E_cov^n, then the node tensor from (D^n, B^n); the state
 * is left exactly as the push of or_sim_step sees it. */
void or_sim_prepare_push(or_sim *s)
{
    field_b_to_n(s);
    compute_nodes(s);
}

/* Deposit the current of moves x1 -> x2 for n test particles (zeroes J). */
void or_sim_deposit_moves(or_sim *s, int64_t n, const double *x1, const double *x2, const double *Q)
{
    for (int c = 0; c < 3; c++) memset(s->J[c], 0, s->gsize * sizeof(double));
    for (int64_t i = 0; i < n; i++) {
        double a[3] = {x1[i], x1[n + i], x1[2 * n + i]};
        double b[3] = {x2[i], x2[n + i], x2[2 * n + i]};
        deposit_particle(s, a, b, Q[i]);
    }
}

/* Trilinear node charge of the given points into out (ghosted layout). */
void or_charge_density(const or_params *p, int64_t n, const double *x, const double *Q, double *out)
{
    size_t gs = (size_t)(p->nx + 3) * (p->ny + 3) * (p->nz + 3);
    memset(out, 0, gs * sizeof(double));
    for (int64_t i = 0; i < n; i++) {
        double X[3] = {x[i], x[n + i], x[2 * n + i]};
        deposit_charge(p, out, X, Q[i]);
    }
}

/* One full cycle (Sec. 2.2 and the ordering at the top of Sec. 3):
 * the state enters as (D^n, B^{n-1/2}, x_n, u_n);
 *   B -> B^n (half-step) with E_cov^n made consistent with B^n by
 *     field_iters fixed-point passes (field_b_to_n);
 *   node tensor from (D^n, B^n);  push x_n -> x_{n+1};
 *   B -> B^{n+1/2} (second half-step with the same E_cov^n);
 *   deposit J^{n+1/2} from the chords;
 *   D -> D^{n+1} with H made consistent with D^{n+1/2} by the same passes
 *     (field_d_step);  relaxation layers;
 *   remove particles inside r_rm or outside the grid.
 * reading: with field_iters = 1 the constitutive coupling is the explicit
 * lag of the printed ordering; the default three passes centre it in time
 * (see the comment above field_b_to_n). */
void or_sim_step(or_sim *s, int nsteps)
{
    const or_params *p = &s->p;
    for (int st = 0; st < nsteps; st++) {
        field_b_to_n(s);
        compute_nodes(s);
        for (int64_t i = 0; i < s->n; i++)
            for (int ax = 0; ax < 3; ax++) s->xold[ax * s->ncap + i] = s->x[ax * s->ncap + i];
        for (int64_t i = 0; i < s->n; i++) {
            if (s->sp[i] == OR_DEAD) continue;
            int sp = s->sp[i];
            double qm = p->mass[sp] != 0.0 ? p->charge[sp] / p->mass[sp] : 0.0;
            double X[3], U[4];
            for (int ax = 0; ax < 3; ax++) X[ax] = s->x[ax * s->ncap + i];
            for (int c = 0; c < 4; c++) U[c] = s->u[c * s->ncap + i];
            push_step(p, s->node, qm, X, U, &s->gamma_clamps);
            for (int ax = 0; ax < 3; ax++) s->x[ax * s->ncap + i] = X[ax];
            for (int c = 0; c < 4; c++) s->u[c * s->ncap + i] = U[c];
        }
        b_half_step(s);
        for (int c = 0; c < 3; c++) memset(s->J[c], 0, s->gsize * sizeof(double));
        for (int64_t i = 0; i < s->n; i++) {
            if (s->sp[i] == OR_DEAD) continue;
            double a[3], b[3];
            for (int ax = 0; ax < 3; ax++) {
                a[ax] = s->xold[ax * s->ncap + i];
                b[ax] = s->x[ax * s->ncap + i];
            }
            deposit_particle(s, a, b, p->charge[s->sp[i]]);
        }
        field_d_step(s);
        relax_inner(s);
        relax_outer(s);
        for (int64_t i = 0; i < s->n; i++) {
            if (s->sp[i] == OR_DEAD) continue;
            double X[3];
            for (int ax = 0; ax < 3; ax++) X[ax] = s->x[ax * s->ncap + i];
            double r = or_radius(p->a, X[0] - p->center[0], X[1] - p->center[1],
                                 X[2] - p->center[2]);
            if (r < p->r_rm) {
                deposit_charge(p, s->rho_abs, X, p->charge[s->sp[i]]);
                s->sp[i] = OR_DEAD;
                s->n_removed_horizon++;
            } else if (outside_grid(p, X)) {
                s->sp[i] = OR_DEAD;
                s->n_removed_outer++;
            }
        }
    }
}

/* Cell key (reading: the paper has no sort; tile edge T).  Tiles of T^3
 * cells are ranked along a boustrophedon path, so consecutive tiles share a
 * face: the planes tz in order; within plane tz the rows ty ascend when tz is
 * even and descend when it is odd; along the r-th row visited (r = tz nTy +
 * the row's place in its plane) the tiles tx ascend when r is even and
 * descend when it is odd.  The path leaves a tile along its row, or, for the
 * last tile of a row, towards the next row (along y, in the plane's row
 * direction), or, for the last tile of a plane, towards the next plane (+z).
 * Inside a tile the cells are numbered in T layers across that exit axis,
 * counted from the side facing away from the exit (the exit side last);
 * within a layer the larger of the two remaining axes is the slow index and
 * the smaller the fast one:
 *   key = rank * T^3 + (layer*T + slow)*T + fast,  (i,j,k) = floor(X);
 * dead particles get 0xFFFFFFFF. */
void or_sort_keys(const or_params *p, int tile, int64_t n, const double *x, const uint8_t *sp,
                  uint32_t *keys)
{
    int T = tile;
    int nTx = (p->nx + T - 1) / T, nTy = (p->ny + T - 1) / T;
    for (int64_t i = 0; i < n; i++) {
        if (sp[i] == OR_DEAD) {
            keys[i] = 0xFFFFFFFFu;
            continue;
        }
        int c[3], t[3], l[3];
        for (int ax = 0; ax < 3; ax++) {
            c[ax] = (int)floor(x[ax * n + i]);
            t[ax] = c[ax] / T;
            l[ax] = c[ax] % T;
        }
        int row_in_plane = (t[2] % 2 == 0) ? t[1] : nTy - 1 - t[1];
        int row = t[2] * nTy + row_in_plane;
        int along = (row % 2 == 0) ? t[0] : nTx - 1 - t[0];
        uint32_t rank = (uint32_t)row * (uint32_t)nTx + (uint32_t)along;
        int exit_axis, exit_up;
        if (along < nTx - 1) {
            exit_axis = 0;
            exit_up = (row % 2 == 0);
        } else if (row_in_plane < nTy - 1) {
            exit_axis = 1;
            exit_up = (t[2] % 2 == 0);
        } else {
            exit_axis = 2;
            exit_up = 1;
        }
        int layer = exit_up ? l[exit_axis] : T - 1 - l[exit_axis];
        int fast = (exit_axis == 0) ? l[1] : l[0];
        int slow = (exit_axis == 2) ? l[1] : l[2];
        keys[i] = rank * (uint32_t)(T * T * T) + (uint32_t)((layer * T + slow) * T + fast);
    }
}

/* Stable order by key: perm[r] = index of the particle of rank r.  A
 * plain insertion-by-merge sort on (key, index) pairs. */
static uint32_t *g_keys_for_cmp;
static int cmp_key_index(const void *A, const void *B)
{
    int64_t ia = *(const int64_t *)A, ib = *(const int64_t *)B;
    uint32_t ka = g_keys_for_cmp[ia], kb = g_keys_for_cmp[ib];
    if (ka != kb) return ka < kb ? -1 : 1;
    return ia < ib ? -1 : (ia > ib ? 1 : 0);
}

void or_stable_order(int64_t n, uint32_t *keys, int64_t *perm)
{
    for (int64_t i = 0; i < n; i++) perm[i] = i;
    g_keys_for_cmp = keys;
    qsort(perm, (size_t)n, sizeof(int64_t), cmp_key_index);
}

/* Diagnostics (reading; the paper reports none): per-species live counts,
 * total charge, particle Killing energy sum M c (-u_4), L_z = sum M (x u_y -
 * y u_x) with covariant u and hole-relative x, field energy
 * (1/8 pi)[sum_E (-E_cov D) + sum_B (B_cov H)] over in-domain points, the
 * Gauss residual max |-div D - 4 pi rho| at interior nodes whose six
 * E points are all updated and outside the relaxation layer, and the
 * mass-shell residual.  Frozen points enter the field energy with the
 * derived values of the reference state.  Pinned: the field energy of m = 0
 * cavity modes equals its closed-form sums; counts, charge, Killing energy
 * and L_z through the conservation tests of the cycle. */
void or_sim_diag(or_sim *s, or_diag *d)
{
    const or_params *p = &s->p;
    memset(d, 0, sizeof(*d));
    double *rho = (double *)calloc(s->gsize, sizeof(double));
    for (int64_t i = 0; i < s->n; i++) {
        if (s->sp[i] == OR_DEAD) continue;
        int sp = s->sp[i];
        d->n_alive[sp]++;
        double X[3], U[4], g[16];
        for (int ax = 0; ax < 3; ax++) X[ax] = s->x[ax * s->ncap + i];
        for (int c = 0; c < 4; c++) U[c] = s->u[c * s->ncap + i];
        d->charge_total += p->charge[sp];
        double x = X[0] - p->center[0], y = X[1] - p->center[1], z = X[2] - p->center[2];
        or_metric(p, x, y, z, g, NULL, NULL);
        double ul[4];
        for (int a = 0; a < 4; a++) {
            double v = 0.0;
            for (int b = 0; b < 4; b++) v += g[a * 4 + b] * U[b];
            ul[a] = v;
        }
        double shell = p->c * p->c;
        for (int a = 0; a < 4; a++) shell += ul[a] * U[a];
        if (fabs(shell) > d->mass_shell_residual_max) d->mass_shell_residual_max = fabs(shell);
        d->energy_particles += p->mass[sp] * p->c * (-ul[3]);
        d->lz_particles += p->mass[sp] * (x * ul[1] - y * ul[0]);
        deposit_charge(p, rho, X, p->charge[sp]);
    }
    compute_Ecov(s);
    compute_H(s);
    double ef = 0.0, bf = 0.0;
    for (int c = 0; c < 3; c++)
        for (int k = 0; k <= p->nz; k++)
            for (int j = 0; j <= p->ny; j++)
                for (int i = 0; i <= p->nx; i++) {
                    size_t id = gidx(p, i, j, k);
                    if (in_domain(p, 0, c, i, j, k)) ef += -s->E[c][id] * s->D[c][id];
                    if (in_domain(p, 1, c, i, j, k)) bf += s->B[c][id] * s->H[c][id];
                }
    d->energy_field = (ef + bf) / (8.0 * M_PI);
    for (int k = 1; k <= p->nz - 1; k++)
        for (int j = 1; j <= p->ny - 1; j++)
            for (int i = 1; i <= p->nx - 1; i++) {
                int ok = 1;
                for (int c = 0; c < 3 && ok; c++) {
                    int im[3] = {i, j, k};
                    im[c] -= 1;
                    if (!updated(p, 0, c, i, j, k) || !updated(p, 0, c, im[0], im[1], im[2]) ||
                        relaxed(p, 0, c, i, j, k) || relaxed(p, 0, c, im[0], im[1], im[2]) ||
                        in_outer_layer(p, 0, c, i, j, k) || in_outer_layer(p, 0, c, im[0], im[1], im[2]))
                        ok = 0;
                }
                if (!ok) continue;
                double div = 0.0;
                for (int c = 0; c < 3; c++) {
                    int im[3] = {i, j, k};
                    im[c] -= 1;
                    div += s->D[c][gidx(p, i, j, k)] - s->D[c][gidx(p, im[0], im[1], im[2])];
                }
                size_t id = gidx(p, i, j, k);
                double res = fabs(-div - 4.0 * M_PI * (rho[id] + s->rho_abs[id]));
                if (res > d->gauss_residual_max) d->gauss_residual_max = res;
            }
    free(rho);
    d->n_removed_horizon = s->n_removed_horizon;
    d->n_removed_outer = s->n_removed_outer;
    d->gamma_clamps = s->gamma_clamps;
    d->flags = s->flags;
}
