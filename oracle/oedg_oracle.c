/*
 * Plain FP64 reference of one BP RI-OEDG step for the 2D Euler equations on
 * triangles (Ding, Cui and Wu, arXiv 2409.09620).  TEST INFRASTRUCTURE ONLY:
 * only the test suite, the smoke check and the benchmark's CPU-baseline leg may
 * load this library.  It shares no code, header or table with the HIP library.
 *
 * The code follows the paper's order and notation, cell by cell, with no
 * blocking or fusion:
 *   mesh notation and affine map ............ Sec. 2 (Fig. MeshK), J_K below eq. basisfunc
 *   orthogonal basis Psi^(0..5) .............. eq. basisfunc
 *   mass a_K^(l) = int_K Psi^2 ............... below eq. DGScalar:Dis (computed by quadrature)
 *   volume / edge quadrature ................. App. A tab:2th, tab:4th, tab:6th; App. B
 *   semi-discrete DG operator L(u) ........... eq. DGSystem:Dis with the LF flux eq. fluxLF
 *   Euler flux and spectral radius ........... Example ex:euler (eq. euler)
 *   SSP-RK3 ................................... eq. RKTime
 *   OE / RIOE filter ......................... eq. oe:sys, OEScalar:Coef1/beta/Coef2,
 *                                              normOmg, oe:sysdelta2, RIOESys:CoefM/Coef1/Coef2
 *   optimal convex decomposition ............. eq. 1040 (P1), eq. 1139 with eq. 1703 (P2)
 *   BP limiter ............................... Sec. 4.4, eqs. 1944 and 1981
 *   BP time step ............................. Sec. 5 (Delta t with C^DCW), eqs. 1692, 1713
 *   classical decomposition (comparison) ..... Sec. 4.2 (Zhang-Xia-Shu weights), the ZXS CFL
 *                                              remarks after eqs. 1692 and 1713, Sec. 4.4
 *                                              (classical branch of the limiter), Sec. 6 Delta t
 *
 * Readings of points the paper leaves open (they are listed in the design notes):
 *   - edge Gauss nodes on [0,1] as s = (1 + x^nu)/2, weights summing to one (App. B);
 *   - the LF viscosity of a stage is the max spectral radius over all edge Gauss
 *     points of that stage's input (eq. 358 / eq. 1250), the step's Delta t uses the
 *     value of u^n;
 *   - beta^(i) uses a guarded spectral radius: rho_s = max(rho, 1e-13), p from rho_s,
 *     sqrt(gamma max(p,0)/rho_s);
 *   - jumps are the neighbour's trace minus the own trace at the same physical
 *     point; on a boundary edge (transmissive or reflective) the jump is zero;
 *   - boundary edges: transmissive (exterior trace = interior trace) or reflective
 *     (exterior trace = interior trace with its normal momentum reversed);
 *   - classical decomposition: the limiter takes the edge Gauss points (P1) or the
 *     edge Gauss points and the vector u* of Sec. 4.4's classical branch, with the
 *     Zhang-Xia-Shu edge weights 2 w1^GL / 3 (P2); its energy bound is E(u*);
 *   - m_n, m_t on both sides use K's own normal n^(i);
 *   - limiter node form: the min runs over the 3Q edge Gauss points plus the P1
 *     vertices v1, v2 (eq. 1944) or the two P2 internal nodes of eq. 1139; the
 *     P2 energy bound is E(u*) of the vector u* (not the printed scalar formula);
 *     optionally (P2) the u* form of Sec. 4.4: edge Gauss points plus the vector
 *     u* formed with the optimal edge weights, energy bound E(u*);
 *   - theta = 1 when the nodal minimum is already >= epsilon (avoids 0/0);
 *   - L-infinity norms use the volume rule's points (eq. normOmg);
 *   - initial data: L2 projection with the 12-point rule (tab:6th), then the BP
 *     limiter, no initial OE.
 *
 * Threads: the cell loops run under OpenMP when it is enabled (orc_set_threads).
 * Each cell's arithmetic is the same on any thread, and every floating-point
 * reduction over cells (domain sums, maxima) is taken serially in cell order, so
 * the results are bit for bit those of one thread.
 */
#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

#define NVAR 4
#define MAXM 6

/* ----------------------------------------------------------------------- constants */

/* App. A, tab:2th: 3-point rule, degree 2. */
static const double TRI3_B[3][3] = {{1.0 / 6, 1.0 / 6, 2.0 / 3}, {1.0 / 6, 2.0 / 3, 1.0 / 6},
                                    {2.0 / 3, 1.0 / 6, 1.0 / 6}};
static const double TRI3_W[3] = {1.0 / 3, 1.0 / 3, 1.0 / 3};

/* App. A, tab:4th: 6-point rule, degree 4.  The printed 15-digit values are the
 * closed forms a = (8 - sqrt(10) + sqrt(38 - 44 sqrt(2/5)))/18,
 * b = (8 - sqrt(10) - sqrt(38 - 44 sqrt(2/5)))/18,
 * w_a,b = (620 +- sqrt(213125 - 53320 sqrt(10)))/3720, evaluated in full precision
 * at set-up. */
static double TRI6_B[6][3], TRI6_W[6];

/* App. A, tab:6th: 12-point rule, degree 6, as printed (used for projection only). */
static const double TRI12_B[12][3] = {
    {0.063089014491502, 0.063089014491502, 0.873821971016996},
    {0.063089014491502, 0.873821971016996, 0.063089014491502},
    {0.873821971016996, 0.063089014491502, 0.063089014491502},
    {0.249286745170910, 0.249286745170910, 0.501426509658180},
    {0.249286745170910, 0.501426509658180, 0.249286745170910},
    {0.501426509658180, 0.249286745170910, 0.249286745170910},
    {0.053145049844817, 0.636502499121399, 0.310352451033784},
    {0.636502499121399, 0.053145049844817, 0.310352451033784},
    {0.053145049844817, 0.310352451033784, 0.636502499121399},
    {0.636502499121399, 0.310352451033784, 0.053145049844817},
    {0.310352451033784, 0.053145049844817, 0.636502499121399},
    {0.310352451033784, 0.636502499121399, 0.053145049844817}};
static const double TRI12_W[12] = {0.050844906370207, 0.050844906370207, 0.050844906370207,
                                   0.116786275726379, 0.116786275726379, 0.116786275726379,
                                   0.082851075618374, 0.082851075618374, 0.082851075618374,
                                   0.082851075618374, 0.082851075618374, 0.082851075618374};

/* App. B: Q = k+1 Gauss-Legendre nodes mapped to s in [0,1], weights sum to 1. */
static double GS[4][3], GW[4][3];

static int consts_ready = 0;
static void init_consts(void) {
    if (consts_ready) return;
    const double r = sqrt(38.0 - 44.0 * sqrt(0.4));
    const double a = (8.0 - sqrt(10.0) + r) / 18.0, b = (8.0 - sqrt(10.0) - r) / 18.0;
    const double q = sqrt(213125.0 - 53320.0 * sqrt(10.0));
    const double wa = (620.0 + q) / 3720.0, wb = (620.0 - q) / 3720.0;
    const double B6[6][3] = {{a, a, 1 - 2 * a}, {a, 1 - 2 * a, a}, {1 - 2 * a, a, a},
                             {b, b, 1 - 2 * b}, {b, 1 - 2 * b, b}, {1 - 2 * b, b, b}};
    for (int m = 0; m < 6; ++m) {
        for (int i = 0; i < 3; ++i) TRI6_B[m][i] = B6[m][i];
        TRI6_W[m] = m < 3 ? wa : wb;
    }
    /* Q = 2: x = -+1/sqrt(3); Q = 3: x = -sqrt(3/5), 0, sqrt(3/5) */
    GS[2][0] = 0.5 * (1.0 - 1.0 / sqrt(3.0));
    GS[2][1] = 0.5 * (1.0 + 1.0 / sqrt(3.0));
    GW[2][0] = GW[2][1] = 0.5;
    GS[3][0] = 0.5 * (1.0 - sqrt(0.6));
    GS[3][1] = 0.5;
    GS[3][2] = 0.5 * (1.0 + sqrt(0.6));
    GW[3][0] = GW[3][2] = 5.0 / 18.0;
    GW[3][1] = 8.0 / 18.0;
    consts_ready = 1;
}

/* ----------------------------------------------------------------------- basis (eq. basisfunc) */

static void basis(double xi, double eta, double* p) {
    p[0] = 1.0;
    p[1] = 4 * xi + 2 * eta - 2;
    p[2] = 3 * eta - 1;
    p[3] = 24 * xi * xi + 24 * xi * eta + 4 * eta * eta - 24 * xi - 8 * eta + 4;
    p[4] = 20 * xi * eta + 10 * eta * eta - 4 * xi - 12 * eta + 2;
    p[5] = 10 * eta * eta - 8 * eta + 1;
}
/* d/dxi and d/deta of the basis */
static void basis_d1(double xi, double eta, double* dx, double* de) {
    dx[0] = 0;                         de[0] = 0;
    dx[1] = 4;                         de[1] = 2;
    dx[2] = 0;                         de[2] = 3;
    dx[3] = 48 * xi + 24 * eta - 24;   de[3] = 24 * xi + 8 * eta - 8;
    dx[4] = 20 * eta - 4;              de[4] = 20 * xi + 20 * eta - 12;
    dx[5] = 0;                         de[5] = 20 * eta - 8;
}
/* second derivatives (xi xi, xi eta, eta eta), constant for P2 */
static void basis_d2(double* xx, double* xe, double* ee) {
    const double a[6] = {0, 0, 0, 48, 0, 0}, b[6] = {0, 0, 0, 24, 20, 0}, c[6] = {0, 0, 0, 8, 20, 20};
    for (int l = 0; l < 6; ++l) { xx[l] = a[l]; xe[l] = b[l]; ee[l] = c[l]; }
}

/* ----------------------------------------------------------------------- Euler (eq. euler) */

typedef struct {
    int k, nm, nc, nq, ne;        /* degree, modes, cells, volume points, edge points */
    int* tri;                      /* nc*3 oriented vertex ids */
    double* vx;                    /* nc*6 oriented vertex coordinates */
    int *nbr, *nbe;                /* nc*3 neighbour cell / its local edge (-1 boundary) */
    double *area, *len, *nrm;      /* nc, nc*3, nc*6 */
    double* jinv;                  /* nc*4: xi_x, xi_y, eta_x, eta_y */
    double* mass;                  /* nc*nm */
    int* perm;                     /* nc*3 local edges sorted by length, descending, stable */
    int* limv;                     /* nc*2 P1: local vertices opposite the two longest edges */
    double* node;                  /* nc*4 P2: internal nodes (x1,y1,x2,y2) */
    double* wdcw;                  /* nc*3 optimal decomposition's edge weights, by local edge */
    double* ck;                    /* nc: C_{K,k} |K| of the active decomposition */
    double *ck_dcw, *ck_zxs;       /* nc: C^DCW_{K,k} |K| and C^ZXS_{K,k} |K| */
    double minck, minck_dcw, minck_zxs, area_sum;
    int* bc;                       /* nc*3: boundary tag of unmatched edges, 0 transmissive, 1 reflective */
    unsigned char* swapped;        /* nc: input vertices 1 and 2 were swapped to orient the cell */
    int zxs;                       /* 1: classical (Zhang-Xia-Shu) decomposition: limiter and Delta t */
    int ustar;                     /* 1: optimal decomposition, P2 limiter in the u* form of Sec. 4.4 */
    /* configuration */
    double gamma, cssp, eps_oe, eps_bp;
    int oe_on, bp_on, oe_mode;     /* oe_mode 0 = rotation invariant, 1 = component-wise */
    /* state, AoS [cell][var][mode] */
    double *u0, *u, *w, *L, *pre;
    double* scratch_c;   /* one double per cell (per-cell maxima before their serial combination) */
    double t, dt, alpha, t_end;
    long step;
    int active, err;
    long n_limited;
    /* step restarts: a stage whose averages leave the admissible set ends the
     * attempt; the step is retried from u^n with half the time step */
    int skip, restarts_this_step, max_restarts;
    long n_restarts;
    /* last stage's globals */
    double ubar[NVAR], nrm_v[NVAR], nrm_m; int zero_v[NVAR], zero_m;
} Orc;

#define U(arr, c, v, l) (arr)[((size_t)(c) * NVAR + (v)) * o->nm + (l)]

static double pressure(const Orc* o, const double* q) {
    return (o->gamma - 1.0) * (q[3] - 0.5 * (q[1] * q[1] + q[2] * q[2]) / q[0]);
}
static double int_energy(const double* q) { return q[3] - 0.5 * (q[1] * q[1] + q[2] * q[2]) / q[0]; }

static void flux(const Orc* o, const double* q, double* f1, double* f2) {
    const double p = pressure(o, q), v1 = q[1] / q[0], v2 = q[2] / q[0];
    f1[0] = q[1]; f1[1] = q[1] * v1 + p; f1[2] = q[2] * v1; f1[3] = (q[3] + p) * v1;
    f2[0] = q[2]; f2[1] = q[1] * v2;     f2[2] = q[2] * v2 + p; f2[3] = (q[3] + p) * v2;
}

/* spectral radius |v.n| + c of F'(u).n, guarded for non-admissible states */
static double spectral_radius(const Orc* o, const double* q, const double* n) {
    const double rs = fmax(q[0], 1e-13);
    const double p = (o->gamma - 1.0) * (q[3] - 0.5 * (q[1] * q[1] + q[2] * q[2]) / rs);
    return fabs(q[1] * n[0] + q[2] * n[1]) / rs + sqrt(o->gamma * fmax(p, 0.0) / rs);
}

/* ----------------------------------------------------------------------- geometry helpers */

static void ref_coords(const Orc* o, int c, double x, double y, double* xi, double* eta) {
    const double* v = o->vx + 6 * c;
    const double* J = o->jinv + 4 * c;
    const double dx = x - v[0], dy = y - v[1];
    *xi = J[0] * dx + J[1] * dy;
    *eta = J[2] * dx + J[3] * dy;
}

static void eval_state(const Orc* o, const double* arr, int c, double xi, double eta, double* q) {
    double p[MAXM];
    basis(xi, eta, p);
    for (int v = 0; v < NVAR; ++v) {
        double s = 0;
        for (int l = 0; l < o->nm; ++l) s += U(arr, c, v, l) * p[l];
        q[v] = s;
    }
}

static void eval_at_xy(const Orc* o, const double* arr, int c, double x, double y, double* q) {
    double xi, eta;
    ref_coords(o, c, x, y, &xi, &eta);
    eval_state(o, arr, c, xi, eta, q);
}

/* local vertex of cell c whose vertex id is vid, or -1 */
static int local_vertex(const Orc* o, int c, int vid) {
    for (int q = 0; q < 3; ++q) if (o->tri[3 * c + q] == vid) return q;
    return -1;
}

/* physical derivatives of every variable at (x,y) in cell c:
 * D[v][0..5] = value, d/dx, d/dy, d2/dx2, d2/dxdy, d2/dy2 */
static void derivs_at_xy(const Orc* o, const double* arr, int c, double x, double y, double D[NVAR][6]) {
    double xi, eta, p[MAXM], dxi[MAXM], deta[MAXM], hxx[MAXM], hxe[MAXM], hee[MAXM];
    ref_coords(o, c, x, y, &xi, &eta);
    basis(xi, eta, p);
    basis_d1(xi, eta, dxi, deta);
    basis_d2(hxx, hxe, hee);
    const double* J = o->jinv + 4 * c;
    const double xx = J[0], xy = J[1], ex = J[2], ey = J[3];
    for (int v = 0; v < NVAR; ++v) {
        double s[6] = {0, 0, 0, 0, 0, 0};
        for (int l = 0; l < o->nm; ++l) {
            const double a = U(arr, c, v, l);
            s[0] += a * p[l];
            s[1] += a * (dxi[l] * xx + deta[l] * ex);
            s[2] += a * (dxi[l] * xy + deta[l] * ey);
            s[3] += a * (hxx[l] * xx * xx + 2 * hxe[l] * xx * ex + hee[l] * ex * ex);
            s[4] += a * (hxx[l] * xx * xy + hxe[l] * (xx * ey + xy * ex) + hee[l] * ex * ey);
            s[5] += a * (hxx[l] * xy * xy + 2 * hxe[l] * xy * ey + hee[l] * ey * ey);
        }
        for (int d = 0; d < 6; ++d) D[v][d] = s[d];
    }
}

/* ----------------------------------------------------------------------- mesh */

typedef struct { int a, b, cell, edge; } EdgeRec;
static int edge_cmp(const void* x, const void* y) {
    const EdgeRec* p = (const EdgeRec*)x;
    const EdgeRec* q = (const EdgeRec*)y;
    if (p->a != q->a) return p->a < q->a ? -1 : 1;
    if (p->b != q->b) return p->b < q->b ? -1 : 1;
    if (p->cell != q->cell) return p->cell < q->cell ? -1 : 1;
    return p->edge < q->edge ? -1 : (p->edge > q->edge);
}

/* Optimal convex decomposition of one triangle with vertices v[0..2] (CCW), edge i
 * opposite vertex i.  Writes the stable descending order of edges, the P1 limiter
 * vertices, the P2 internal nodes and C^DCW_{K,k}.  Eq. 1040 (P1), eq. 1139 + 1703 (P2). */
static void decompose(int k, const double* v, const double* len, int* perm, int* limv,
                      double* node, double* wts, double* node_w, double* cdcw) {
    int p[3] = {0, 1, 2};
    /* stable insertion sort by length, descending */
    for (int i = 1; i < 3; ++i) {
        int x = p[i], j = i - 1;
        while (j >= 0 && len[p[j]] < len[x]) { p[j + 1] = p[j]; --j; }
        p[j + 1] = x;
    }
    for (int i = 0; i < 3; ++i) perm[i] = p[i];
    const double l1 = len[p[0]], l2 = len[p[1]], l3 = len[p[2]];
    const double* V[3] = {v + 2 * p[0], v + 2 * p[1], v + 2 * p[2]};  /* v^(i) opposite e^(i) */
    limv[0] = p[0];
    limv[1] = p[1];
    if (k == 1) {
        for (int i = 0; i < 3; ++i) wts[i] = 2.0 * len[p[i]] / (3.0 * l1 + 3.0 * l2);
        node_w[0] = (l1 + l2 - 2.0 * l3) / (3.0 * l1 + 3.0 * l2);
        node_w[1] = 0.0;
        const double den = l1 + l2 - 2.0 * l3;
        if (den > 0) {
            node[0] = ((l1 - l3) * V[0][0] + (l2 - l3) * V[1][0]) / den;
            node[1] = ((l1 - l3) * V[0][1] + (l2 - l3) * V[1][1]) / den;
        } else {
            node[0] = (V[0][0] + V[1][0] + V[2][0]) / 3.0;
            node[1] = (V[0][1] + V[1][1] + V[2][1]) / 3.0;
        }
        node[2] = node[0];
        node[3] = node[1];
        *cdcw = 2.0 / (3.0 * (l1 + l2));
    } else {
        const double lb = (l1 + l2 + l3) / 3.0;
        const double lh = sqrt(l1 * l1 + l2 * l2 + l3 * l3 - (2.0 / 3.0) * (l1 * l2 + l2 * l3 + l3 * l1));
        const double s3 = sqrt(3.0);
        for (int i = 0; i < 3; ++i) wts[i] = 2.0 * len[p[i]] / (9.0 * lb + 3.0 * lh);
        node_w[0] = node_w[1] = (lb + lh) / (6.0 * lb + 2.0 * lh);
        const double c[2][3] = {
            {3 * l1 + 3 * l2 + s3 * l2 - s3 * l3, 6 * l2 + s3 * l3 - s3 * l1, 3 * l2 + 3 * l3 + s3 * l1 - s3 * l2},
            {3 * l1 + 3 * l2 + s3 * l3 - s3 * l2, 6 * l2 + s3 * l1 - s3 * l3, 3 * l2 + 3 * l3 + s3 * l2 - s3 * l1}};
        const double M[2][3][3][3] = {
            {{{6, 1, -2}, {1, 2 * s3 + 6, -s3 - 2}, {-2, -s3 - 2, 6}},
             {{6, -s3 - 2, -2}, {-s3 - 2, 12, s3 - 2}, {-2, s3 - 2, 6}},
             {{6, s3 - 2, -2}, {s3 - 2, 6 - 2 * s3, 1}, {-2, 1, 6}}},
            {{{6, 1, -2}, {1, 6 - 2 * s3, s3 - 2}, {-2, s3 - 2, 6}},
             {{6, s3 - 2, -2}, {s3 - 2, 12, -s3 - 2}, {-2, -s3 - 2, 6}},
             {{6, -s3 - 2, -2}, {-s3 - 2, 2 * s3 + 6, 1}, {-2, 1, 6}}}};
        const double lv[3] = {l1, l2, l3};
        const double den = 18.0 * (lb + lh) * (l2 + lh);
        for (int s = 0; s < 2; ++s) {
            double x = 0, y = 0;
            for (int i = 0; i < 3; ++i) {
                double quad = 0;
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) quad += lv[a] * M[s][i][a][b] * lv[b];
                const double beta = (quad + 2.0 * c[s][i] * lh) / den;
                x += beta * V[i][0];
                y += beta * V[i][1];
            }
            node[2 * s] = x;
            node[2 * s + 1] = y;
        }
        *cdcw = 2.0 / (9.0 * lb + 3.0 * lh);
    }
}

/* exported for the decomposition pins: one triangle, weights in the sorted edge
 * order (w_1 >= w_2 >= w_3 correspond to l_1 >= l_2 >= l_3) */
int orc_decompose(int k, const double* v, double* wts, double* nodes, double* node_w, double* cdcw,
                  int* perm) {
    double len[3];
    int limv[2];
    for (int i = 0; i < 3; ++i) {
        const double* a = v + 2 * ((i + 1) % 3);
        const double* b = v + 2 * ((i + 2) % 3);
        const double dx = b[0] - a[0], dy = b[1] - a[1];
        len[i] = sqrt(dx * dx + dy * dy);
    }
    decompose(k, v, len, perm, limv, nodes, wts, node_w, cdcw);
    return 0;
}

static void* xcalloc(size_t n, size_t s) { return calloc(n ? n : 1, s); }

void orc_destroy(Orc* o) {
    if (!o) return;
    free(o->tri); free(o->vx); free(o->nbr); free(o->nbe); free(o->area); free(o->len);
    free(o->nrm); free(o->jinv); free(o->mass); free(o->perm); free(o->limv); free(o->node); free(o->wdcw);
    free(o->ck); free(o->ck_dcw); free(o->ck_zxs); free(o->bc); free(o->swapped); free(o->u0); free(o->u); free(o->w); free(o->L); free(o->pre);
    free(o->scratch_c);
    free(o);
}

/* Build the mesh: orientation, edge table (edge i opposite vertex i runs from
 * vertex i+1 to vertex i+2), geometry, decomposition and the mass matrix. */
Orc* orc_create(int k, int nv, const double* xy, int nc, const int* tri_in, const double* cell_xy) {
    init_consts();
    if (k < 1 || k > 2 || nc < 0 || nv < 0) return NULL;
    Orc* o = (Orc*)xcalloc(1, sizeof(Orc));
    o->k = k;
    o->nm = (k + 1) * (k + 2) / 2;
    o->nc = nc;
    o->nq = k == 1 ? 3 : 6;
    o->ne = k + 1;
    o->gamma = 1.4;
    o->cssp = 1.0;
    o->max_restarts = 8;
    o->eps_oe = 1e-12;
    o->eps_bp = 1e-13;
    o->oe_on = 1;
    o->bp_on = 1;
    o->t_end = INFINITY;
    o->tri = (int*)xcalloc((size_t)nc * 3, sizeof(int));
    o->vx = (double*)xcalloc((size_t)nc * 6, sizeof(double));
    o->nbr = (int*)xcalloc((size_t)nc * 3, sizeof(int));
    o->nbe = (int*)xcalloc((size_t)nc * 3, sizeof(int));
    o->area = (double*)xcalloc(nc, sizeof(double));
    o->len = (double*)xcalloc((size_t)nc * 3, sizeof(double));
    o->nrm = (double*)xcalloc((size_t)nc * 6, sizeof(double));
    o->jinv = (double*)xcalloc((size_t)nc * 4, sizeof(double));
    o->mass = (double*)xcalloc((size_t)nc * o->nm, sizeof(double));
    o->perm = (int*)xcalloc((size_t)nc * 3, sizeof(int));
    o->limv = (int*)xcalloc((size_t)nc * 2, sizeof(int));
    o->node = (double*)xcalloc((size_t)nc * 4, sizeof(double));
    o->wdcw = (double*)xcalloc((size_t)nc * 3, sizeof(double));
    o->ck = (double*)xcalloc(nc, sizeof(double));
    o->ck_dcw = (double*)xcalloc(nc, sizeof(double));
    o->ck_zxs = (double*)xcalloc(nc, sizeof(double));
    o->bc = (int*)xcalloc((size_t)nc * 3, sizeof(int));
    o->swapped = (unsigned char*)xcalloc(nc, 1);
    const size_t ns = (size_t)nc * NVAR * o->nm;
    o->u0 = (double*)xcalloc(ns, sizeof(double));
    o->u = (double*)xcalloc(ns, sizeof(double));
    o->w = (double*)xcalloc(ns, sizeof(double));
    o->L = (double*)xcalloc(ns, sizeof(double));
    o->pre = (double*)xcalloc(ns, sizeof(double));
    o->scratch_c = (double*)xcalloc((size_t)o->nc, sizeof(double));

    /* coordinates and counter-clockwise orientation */
    for (int c = 0; c < nc; ++c) {
        double v[6];
        int id[3];
        for (int q = 0; q < 3; ++q) {
            id[q] = tri_in[3 * c + q];
            if (id[q] < 0 || id[q] >= nv) { orc_destroy(o); return NULL; }
            if (cell_xy) { v[2 * q] = cell_xy[6 * c + 2 * q]; v[2 * q + 1] = cell_xy[6 * c + 2 * q + 1]; }
            else { v[2 * q] = xy[2 * id[q]]; v[2 * q + 1] = xy[2 * id[q] + 1]; }
        }
        const double det = (v[2] - v[0]) * (v[5] - v[1]) - (v[4] - v[0]) * (v[3] - v[1]);
        if (det == 0.0) { orc_destroy(o); return NULL; }
        if (det < 0) {  /* swap vertices 1 and 2 */
            o->swapped[c] = 1;
            int ti = id[1]; id[1] = id[2]; id[2] = ti;
            double tx = v[2], ty = v[3];
            v[2] = v[4]; v[3] = v[5]; v[4] = tx; v[5] = ty;
        }
        for (int q = 0; q < 3; ++q) o->tri[3 * c + q] = id[q];
        for (int q = 0; q < 6; ++q) o->vx[6 * c + q] = v[q];
    }

    /* edge table by sorting (min id, max id) keys */
    EdgeRec* E = (EdgeRec*)xcalloc((size_t)nc * 3, sizeof(EdgeRec));
    for (int c = 0; c < nc; ++c)
        for (int i = 0; i < 3; ++i) {
            const int a = o->tri[3 * c + (i + 1) % 3], b = o->tri[3 * c + (i + 2) % 3];
            EdgeRec* e = &E[3 * c + i];
            e->a = a < b ? a : b;
            e->b = a < b ? b : a;
            e->cell = c;
            e->edge = i;
            o->nbr[3 * c + i] = -1;
            o->nbe[3 * c + i] = -1;
        }
    qsort(E, (size_t)nc * 3, sizeof(EdgeRec), edge_cmp);
    for (size_t i = 0; i + 1 < (size_t)nc * 3; ++i) {
        if (E[i].a == E[i + 1].a && E[i].b == E[i + 1].b) {
            if (i + 2 < (size_t)nc * 3 && E[i + 2].a == E[i].a && E[i + 2].b == E[i].b) {
                free(E); orc_destroy(o); return NULL;   /* non-manifold edge */
            }
            o->nbr[3 * E[i].cell + E[i].edge] = E[i + 1].cell;
            o->nbe[3 * E[i].cell + E[i].edge] = E[i + 1].edge;
            o->nbr[3 * E[i + 1].cell + E[i + 1].edge] = E[i].cell;
            o->nbe[3 * E[i + 1].cell + E[i + 1].edge] = E[i].edge;
            ++i;
        }
    }
    free(E);

    /* geometry: |K|, lengths, outward normals, J^{-1}; decomposition; mass */
    o->minck_dcw = o->minck_zxs = INFINITY;
    o->area_sum = 0;
    for (int c = 0; c < nc; ++c) {
        const double* v = o->vx + 6 * c;
        const double j11 = v[2] - v[0], j12 = v[4] - v[0], j21 = v[3] - v[1], j22 = v[5] - v[1];
        const double det = j11 * j22 - j12 * j21;
        o->area[c] = 0.5 * det;
        o->area_sum += o->area[c];
        double* J = o->jinv + 4 * c;
        J[0] = j22 / det;  J[1] = -j12 / det;  /* xi_x, xi_y */
        J[2] = -j21 / det; J[3] = j11 / det;   /* eta_x, eta_y */
        for (int i = 0; i < 3; ++i) {
            const double* a = v + 2 * ((i + 1) % 3);
            const double* b = v + 2 * ((i + 2) % 3);
            const double dx = b[0] - a[0], dy = b[1] - a[1];
            const double l = sqrt(dx * dx + dy * dy);
            o->len[3 * c + i] = l;
            o->nrm[6 * c + 2 * i] = dy / l;      /* CCW: outward normal is (dy, -dx)/l */
            o->nrm[6 * c + 2 * i + 1] = -dx / l;
        }
        double wts[3], nw[2], cd;
        decompose(k, v, o->len + 3 * c, o->perm + 3 * c, o->limv + 2 * c, o->node + 4 * c, wts, nw, &cd);
        for (int i = 0; i < 3; ++i) o->wdcw[3 * c + o->perm[3 * c + i]] = wts[i];
        o->ck_dcw[c] = cd * o->area[c];
        if (o->ck_dcw[c] < o->minck_dcw) o->minck_dcw = o->ck_dcw[c];
        /* classical decomposition: C^ZXS = 1/(9 lbar) (P1), 1/(27 lbar) (P2), lbar the
         * mean edge length (remarks after eqs. 1692 and 1713) */
        const double lbar = (o->len[3 * c] + o->len[3 * c + 1] + o->len[3 * c + 2]) / 3.0;
        o->ck_zxs[c] = o->area[c] / ((k == 1 ? 9.0 : 27.0) * lbar);
        if (o->ck_zxs[c] < o->minck_zxs) o->minck_zxs = o->ck_zxs[c];
        /* a_K^(l) = int_K Psi_l^2, exact with the degree-4 rule */
        for (int l = 0; l < o->nm; ++l) {
            double s = 0;
            for (int m = 0; m < 6; ++m) {
                double p[MAXM];
                basis(TRI6_B[m][1], TRI6_B[m][2], p);
                s += TRI6_W[m] * p[l] * p[l];
            }
            o->mass[(size_t)c * o->nm + l] = o->area[c] * s;
        }
    }
    memcpy(o->ck, o->ck_dcw, sizeof(double) * nc);
    o->minck = o->minck_dcw;
    o->active = 1;
    return o;
}

/* boundary tags of the unmatched edges: tags[3c+i] for the edge of cell c opposite
 * its input vertex i (entries of matched edges are ignored); 0 transmissive,
 * 1 reflective.  Orienting a cell swaps its vertices 1 and 2, and so its edges 1
 * and 2. */
int orc_set_bc(Orc* o, const int* tags) {
    for (int c = 0; c < o->nc; ++c)
        for (int i = 0; i < 3; ++i) {
            const int in = o->swapped[c] && i > 0 ? 3 - i : i;
            const int t = tags ? tags[3 * c + in] : 0;
            if (o->nbr[3 * c + i] >= 0) { o->bc[3 * c + i] = 0; continue; }
            if (t != 0 && t != 1) return -1;
            o->bc[3 * c + i] = t;
        }
    return 0;
}

/* 0: the optimal decomposition (DCW), 1: the classical one (ZXS), for the limiter
 * and the time step; call before the initial state is set */
/* limiter form of the optimal decomposition: 0 the node form, 1 the u* form of
 * Sec. 4.4 (differs for P2 only) */
int orc_set_limiter_form(Orc* o, int ustar) {
    if (ustar != 0 && ustar != 1) return -1;
    o->ustar = ustar;
    return 0;
}

int orc_set_decomp(Orc* o, int zxs) {
    if (zxs != 0 && zxs != 1) return -1;
    o->zxs = zxs;
    memcpy(o->ck, zxs ? o->ck_zxs : o->ck_dcw, sizeof(double) * o->nc);
    o->minck = zxs ? o->minck_zxs : o->minck_dcw;
    return 0;
}

int orc_export_mesh(const Orc* o, int* tri, int* nbr, int* nbe, int* perm, int* limv, double* area,
                    double* len, double* nrm, double* node, double* ck, double* minck) {
    const int nc = o->nc;
    if (tri) memcpy(tri, o->tri, sizeof(int) * 3 * nc);
    if (nbr) memcpy(nbr, o->nbr, sizeof(int) * 3 * nc);
    if (nbe) memcpy(nbe, o->nbe, sizeof(int) * 3 * nc);
    if (perm) memcpy(perm, o->perm, sizeof(int) * 3 * nc);
    if (limv) memcpy(limv, o->limv, sizeof(int) * 2 * nc);
    if (area) memcpy(area, o->area, sizeof(double) * nc);
    if (len) memcpy(len, o->len, sizeof(double) * 3 * nc);
    if (nrm) memcpy(nrm, o->nrm, sizeof(double) * 6 * nc);
    if (node) memcpy(node, o->node, sizeof(double) * 4 * nc);
    if (ck) memcpy(ck, o->ck, sizeof(double) * nc);
    if (minck) *minck = o->minck;
    return 0;
}

int orc_config(Orc* o, double gamma, double cssp, int oe_on, int bp_on, int oe_mode) {
    o->gamma = gamma;
    o->cssp = cssp;
    o->oe_on = oe_on;
    o->bp_on = bp_on;
    o->oe_mode = oe_mode;
    return 0;
}

/* ----------------------------------------------------------------------- L(u) */

/* eq. DGSystem:Dis: a^(l) du^(l)/dt = |K| sum_mu w_mu F(u).grad Psi - sum_i l_i sum_nu w_nu Fhat Psi */
static void residual(Orc* o, const double* arr, double alpha, double* Lout) {
    const int nm = o->nm, Q = o->ne;
    const double(*VB)[3] = o->k == 1 ? TRI3_B : (const double(*)[3])TRI6_B;
    const double* VW = o->k == 1 ? TRI3_W : TRI6_W;
#pragma omp parallel for schedule(static)
    for (int c = 0; c < o->nc; ++c) {
        double rhs[NVAR][MAXM];
        memset(rhs, 0, sizeof(rhs));
        const double* J = o->jinv + 4 * c;
        /* volume integral */
        for (int m = 0; m < o->nq; ++m) {
            const double xi = VB[m][1], eta = VB[m][2];
            double q[NVAR], f1[NVAR], f2[NVAR], dxi[MAXM], deta[MAXM];
            eval_state(o, arr, c, xi, eta, q);
            flux(o, q, f1, f2);
            basis_d1(xi, eta, dxi, deta);
            for (int l = 1; l < nm; ++l) {
                const double gx = dxi[l] * J[0] + deta[l] * J[2];
                const double gy = dxi[l] * J[1] + deta[l] * J[3];
                for (int v = 0; v < NVAR; ++v)
                    rhs[v][l] += o->area[c] * VW[m] * (f1[v] * gx + f2[v] * gy);
            }
        }
        /* surface integral with the LF flux */
        const double* vc = o->vx + 6 * c;
        for (int i = 0; i < 3; ++i) {
            const int la = (i + 1) % 3, lb = (i + 2) % 3;
            const double* pa = vc + 2 * la;
            const double* pb = vc + 2 * lb;
            const int nb = o->nbr[3 * c + i];
            const double* n = o->nrm + 6 * c + 2 * i;
            int qa = -1, qb = -1;
            if (nb >= 0) {
                qa = local_vertex(o, nb, o->tri[3 * c + la]);
                qb = local_vertex(o, nb, o->tri[3 * c + lb]);
            }
            for (int g = 0; g < Q; ++g) {
                const double s = GS[Q][g];
                const double x = pa[0] + s * (pb[0] - pa[0]), y = pa[1] + s * (pb[1] - pa[1]);
                double xi, eta, p[MAXM], qi[NVAR], qe[NVAR];
                ref_coords(o, c, x, y, &xi, &eta);
                basis(xi, eta, p);
                eval_state(o, arr, c, xi, eta, qi);
                if (nb >= 0) {
                    const double* vn = o->vx + 6 * nb;
                    const double xn = vn[2 * qa] + s * (vn[2 * qb] - vn[2 * qa]);
                    const double yn = vn[2 * qa + 1] + s * (vn[2 * qb + 1] - vn[2 * qa + 1]);
                    eval_at_xy(o, arr, nb, xn, yn, qe);
                } else if (o->bc[3 * c + i] == 1) {
                    /* reflective wall: the normal momentum reversed */
                    const double mn = qi[1] * n[0] + qi[2] * n[1];
                    qe[0] = qi[0];
                    qe[1] = qi[1] - 2.0 * mn * n[0];
                    qe[2] = qi[2] - 2.0 * mn * n[1];
                    qe[3] = qi[3];
                } else {
                    for (int v = 0; v < NVAR; ++v) qe[v] = qi[v];
                }
                double f1i[NVAR], f2i[NVAR], f1e[NVAR], f2e[NVAR];
                flux(o, qi, f1i, f2i);
                flux(o, qe, f1e, f2e);
                for (int v = 0; v < NVAR; ++v) {
                    const double fh = 0.5 * (f1i[v] * n[0] + f2i[v] * n[1] + f1e[v] * n[0] + f2e[v] * n[1]
                                             - alpha * (qe[v] - qi[v]));
                    for (int l = 0; l < nm; ++l) rhs[v][l] -= o->len[3 * c + i] * GW[Q][g] * fh * p[l];
                }
            }
        }
        for (int v = 0; v < NVAR; ++v)
            for (int l = 0; l < nm; ++l) U(Lout, c, v, l) = rhs[v][l] / o->mass[(size_t)c * nm + l];
    }
}

/* ----------------------------------------------------------------------- max wave speed */

/* eq. 1250: alpha = max over every cell, edge and edge Gauss point of R(u_h, n) */
static double max_wave_speed(const Orc* o, const double* arr) {
    const int Q = o->ne;
    double* rc = o->scratch_c;   /* the cells' own maxima, then combined in cell order */
#pragma omp parallel for schedule(static)
    for (int c = 0; c < o->nc; ++c) {
        const double* vc = o->vx + 6 * c;
        double a = 0;
        for (int i = 0; i < 3; ++i) {
            const double* pa = vc + 2 * ((i + 1) % 3);
            const double* pb = vc + 2 * ((i + 2) % 3);
            for (int g = 0; g < Q; ++g) {
                const double s = GS[Q][g];
                double q[NVAR];
                eval_at_xy(o, arr, c, pa[0] + s * (pb[0] - pa[0]), pa[1] + s * (pb[1] - pa[1]), q);
                const double r = spectral_radius(o, q, o->nrm + 6 * c + 2 * i);
                if (r > a || r != r) a = r;
            }
        }
        rc[c] = a;
    }
    double a = 0;
    for (int c = 0; c < o->nc; ++c)
        if (rc[c] > a || rc[c] != rc[c]) a = rc[c];
    return a;
}

/* ----------------------------------------------------------------------- OE (Sec. 3) */

static double A_kj(int k, int j) {
    double f = 1;
    for (int i = 2; i <= j; ++i) f *= i;
    return (2.0 * j + 1.0) / ((2.0 * k - 1.0) * f);
}

/* 0.5 sum_{|alpha|=j} C_j^{alpha_1} (jump_c^2 + jump_d^2) for one scalar field whose
 * jumps of (value, dx, dy, dxx, dxy, dyy) at the two endpoints are jc and jd */
static double jump_energy(int j, const double* jc, const double* jd) {
    if (j == 0) return 0.5 * (jc[0] * jc[0] + jd[0] * jd[0]);
    if (j == 1) return 0.5 * (jc[1] * jc[1] + jc[2] * jc[2] + jd[1] * jd[1] + jd[2] * jd[2]);
    return 0.5 * (jc[3] * jc[3] + 2.0 * jc[4] * jc[4] + jc[5] * jc[5] +
                  jd[3] * jd[3] + 2.0 * jd[4] * jd[4] + jd[5] * jd[5]);
}

static void oe_filter(Orc* o, double* arr, double dt) {
    const int nm = o->nm, k = o->k;
    const double(*VB)[3] = o->k == 1 ? TRI3_B : (const double(*)[3])TRI6_B;
    /* domain averages (sum of |K| ubar_K / |Omega|), eq. below OEScalar:Coef2 */
    double sA[NVAR] = {0, 0, 0, 0};
    for (int c = 0; c < o->nc; ++c)
        for (int v = 0; v < NVAR; ++v) sA[v] += o->area[c] * U(arr, c, v, 0);
    for (int v = 0; v < NVAR; ++v) o->ubar[v] = sA[v] / o->area_sum;
    /* L-infinity norms at the volume points, eq. normOmg */
    double nv[NVAR] = {0, 0, 0, 0}, nmv = 0;
    for (int c = 0; c < o->nc; ++c)
        for (int m = 0; m < o->nq; ++m) {
            double q[NVAR];
            eval_state(o, arr, c, VB[m][1], VB[m][2], q);
            for (int v = 0; v < NVAR; ++v) nv[v] = fmax(nv[v], fabs(q[v] - o->ubar[v]));
            const double d1 = q[1] - o->ubar[1], d2 = q[2] - o->ubar[2];
            nmv = fmax(nmv, sqrt(d1 * d1 + d2 * d2));
        }
    for (int v = 0; v < NVAR; ++v) {
        o->nrm_v[v] = nv[v];
        o->zero_v[v] = nv[v] <= o->eps_oe * fmax(1.0, fabs(o->ubar[v]));
    }
    o->nrm_m = nmv;
    o->zero_m = nmv <= o->eps_oe * fmax(1.0, sqrt(o->ubar[1] * o->ubar[1] + o->ubar[2] * o->ubar[2]));

    double* out = o->L;  /* scratch: damped copy, so every cell sees the unfiltered field */
    memcpy(out, arr, sizeof(double) * (size_t)o->nc * NVAR * nm);
#pragma omp parallel for schedule(dynamic, 64)
    for (int c = 0; c < o->nc; ++c) {
        double sigma[NVAR][3];
        memset(sigma, 0, sizeof(sigma));
        for (int i = 0; i < 3; ++i) {
            const int nb = o->nbr[3 * c + i];
            if (nb < 0) continue;   /* boundary edge (transmissive or reflective): zero jump */
            const int la = (i + 1) % 3, lb = (i + 2) % 3;
            const int qa = local_vertex(o, nb, o->tri[3 * c + la]);
            const int qb = local_vertex(o, nb, o->tri[3 * c + lb]);
            const double* n = o->nrm + 6 * c + 2 * i;
            const double* vc = o->vx + 6 * c;
            const double* vn = o->vx + 6 * nb;
            double Dc[NVAR][6], Dcn[NVAR][6], Dd[NVAR][6], Ddn[NVAR][6];
            derivs_at_xy(o, arr, c, vc[2 * la], vc[2 * la + 1], Dc);
            derivs_at_xy(o, arr, nb, vn[2 * qa], vn[2 * qa + 1], Dcn);
            derivs_at_xy(o, arr, c, vc[2 * lb], vc[2 * lb + 1], Dd);
            derivs_at_xy(o, arr, nb, vn[2 * qb], vn[2 * qb + 1], Ddn);
            /* beta^(i): max spectral radius at both endpoints, both sides */
            double beta = 0;
            {
                double q[NVAR];
                for (int v = 0; v < NVAR; ++v) q[v] = Dc[v][0];
                beta = fmax(beta, spectral_radius(o, q, n));
                for (int v = 0; v < NVAR; ++v) q[v] = Dcn[v][0];
                beta = fmax(beta, spectral_radius(o, q, n));
                for (int v = 0; v < NVAR; ++v) q[v] = Dd[v][0];
                beta = fmax(beta, spectral_radius(o, q, n));
                for (int v = 0; v < NVAR; ++v) q[v] = Ddn[v][0];
                beta = fmax(beta, spectral_radius(o, q, n));
            }
            /* jumps (neighbour minus own) of every derivative */
            double jc[NVAR][6], jd[NVAR][6], jcn[6], jdn[6], jct[6], jdt[6];
            for (int v = 0; v < NVAR; ++v)
                for (int d = 0; d < 6; ++d) {
                    jc[v][d] = Dcn[v][d] - Dc[v][d];
                    jd[v][d] = Ddn[v][d] - Dd[v][d];
                }
            for (int d = 0; d < 6; ++d) {   /* m_n = m.n, m_t = m.(-n2, n1) */
                jcn[d] = jc[1][d] * n[0] + jc[2][d] * n[1];
                jdn[d] = jd[1][d] * n[0] + jd[2][d] * n[1];
                jct[d] = -jc[1][d] * n[1] + jc[2][d] * n[0];
                jdt[d] = -jd[1][d] * n[1] + jd[2][d] * n[0];
            }
            const double h = 2.0 * o->area[c] / o->len[3 * c + i];
            double hj = 1.0;
            for (int j = 0; j <= k; ++j) {
                const double A = A_kj(k, j);
                double delta[NVAR];
                for (int v = 0; v < NVAR; v += 3)
                    delta[v] = o->zero_v[v] ? 0.0 : A * hj / o->nrm_v[v] * sqrt(jump_energy(j, jc[v], jd[v]));
                if (o->oe_mode == 0) {
                    const double dn = sqrt(jump_energy(j, jcn, jdn)), dtg = sqrt(jump_energy(j, jct, jdt));
                    const double dm = o->zero_m ? 0.0 : A * hj / o->nrm_m * fmax(dn, dtg);
                    delta[1] = delta[2] = dm;
                } else {
                    for (int v = 1; v <= 2; ++v)
                        delta[v] = o->zero_v[v] ? 0.0
                                                : A * hj / o->nrm_v[v] * sqrt(jump_energy(j, jc[v], jd[v]));
                }
                for (int v = 0; v < NVAR; ++v) sigma[v][j] += beta / h * delta[v];
                hj *= h;
            }
        }
        /* exact solution of the damping ODE, eq. oe:sys: degree-m modes times
         * exp(-dt sum_{j<=m} sigma^j), mode 0 untouched (eq. OE:m0) */
        for (int v = 0; v < NVAR; ++v) {
            double acc = sigma[v][0];
            for (int m = 1; m <= k; ++m) {
                acc += sigma[v][m];
                const double f = exp(-dt * acc);
                const int l0 = m * (m + 1) / 2, l1 = (m + 1) * (m + 2) / 2;
                for (int l = l0; l < l1; ++l) U(out, c, v, l) = U(arr, c, v, l) * f;
            }
        }
    }
    memcpy(arr, out, sizeof(double) * (size_t)o->nc * NVAR * nm);
}

/* ----------------------------------------------------------------------- BP limiter (Sec. 4.4) */

/* physical points of the optimal decomposition's limiter node set: 3Q edge Gauss
 * points, then the P1 vertices v1, v2 (eq. 1944) or the two P2 internal nodes
 * (eq. 1139) */
static int limiter_points(const Orc* o, int c, double* px, double* py) {
    const int Q = o->ne;
    const double* vc = o->vx + 6 * c;
    int n = 0;
    for (int i = 0; i < 3; ++i) {
        const double* pa = vc + 2 * ((i + 1) % 3);
        const double* pb = vc + 2 * ((i + 2) % 3);
        for (int g = 0; g < Q; ++g) {
            const double s = GS[Q][g];
            px[n] = pa[0] + s * (pb[0] - pa[0]);
            py[n] = pa[1] + s * (pb[1] - pa[1]);
            ++n;
        }
    }
    if (o->k == 1) {
        for (int t = 0; t < 2; ++t) {
            const int lv = o->limv[2 * c + t];
            px[n] = vc[2 * lv];
            py[n] = vc[2 * lv + 1];
            ++n;
        }
    } else {
        for (int s = 0; s < 2; ++s) {
            px[n] = o->node[4 * c + 2 * s];
            py[n] = o->node[4 * c + 2 * s + 1];
            ++n;
        }
    }
    return n;
}

/* The state at the limiter's node set of cell c, q[t][v], t < 3Q + 2.
 * Optimal decomposition: the points above; in the u* form of Sec. 4.4 (P2 only)
 * the two internal nodes give way to the vector
 *   u* = (ubar - sum_i w_i sum_nu w^G_nu u(x_i,nu)) / (1 - sum_i w_i)
 * with the optimal decomposition's edge weights w_i (eq. 1139), held twice.
 * Classical decomposition (Sec. 4.4,
 * classical branch): the 3Q edge Gauss points, then for P2 the vector
 *   u* = (ubar - sum_i w_i sum_nu w^G_nu u(x_i,nu)) / (1 - sum_i w_i),
 * w_i = 2 w1^GL / 3 with w1^GL = 1/(L(L-1)), L = ceil((k+3)/2) (Sec. 4.2), the
 * average of the internal nodes of that decomposition; P1 has no internal nodes
 * (sum_i w_i = 1).  The two trailing entries repeat edge points 0 and 1 (P1) or
 * hold u* twice (P2), which leaves every minimum unchanged. */
static int limiter_values(const Orc* o, const double* arr, int c, double q[12][NVAR]) {
    double px[12], py[12];
    const int n = limiter_points(o, c, px, py), ne = 3 * o->ne;
    for (int t = 0; t < (o->zxs ? ne : n); ++t) eval_at_xy(o, arr, c, px[t], py[t], q[t]);
    if (!o->zxs) {
        if (o->ustar && o->k == 2) {
            double acc[NVAR] = {0, 0, 0, 0}, wsum = 0.0;
            for (int i = 0; i < 3; ++i) {
                const double wi = o->wdcw[3 * c + i];
                wsum += wi;
                for (int g = 0; g < o->ne; ++g)
                    for (int v = 0; v < NVAR; ++v) acc[v] += wi * GW[o->ne][g] * q[i * o->ne + g][v];
            }
            for (int v = 0; v < NVAR; ++v) q[ne][v] = q[ne + 1][v] = (U(arr, c, v, 0) - acc[v]) / (1.0 - wsum);
        }
        return n;
    }
    if (o->k == 1) {
        for (int v = 0; v < NVAR; ++v) { q[ne][v] = q[0][v]; q[ne + 1][v] = q[1][v]; }
        return n;
    }
    const int L = (o->k + 4) / 2;   /* ceil((k+3)/2) */
    const double w1 = 1.0 / (L * (L - 1)), wi = 2.0 * w1 / 3.0;
    double acc[NVAR] = {0, 0, 0, 0};
    for (int i = 0; i < 3; ++i)
        for (int g = 0; g < o->ne; ++g)
            for (int v = 0; v < NVAR; ++v) acc[v] += wi * GW[o->ne][g] * q[i * o->ne + g][v];
    for (int v = 0; v < NVAR; ++v) {
        const double us = (U(arr, c, v, 0) - acc[v]) / (1.0 - 3.0 * wi);
        q[ne][v] = q[ne + 1][v] = us;
    }
    return n;
}

/* returns the number of cells whose average is not admissible */
static int bp_limit(Orc* o, double* arr) {
    int bad = 0;
    long limited = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad, limited)
    for (int c = 0; c < o->nc; ++c) {
        double q[12][NVAR];
        /* step 1: density */
        const int np = limiter_values(o, arr, c, q);
        const double rb = U(arr, c, 0, 0);
        double rmin = INFINITY;
        for (int t = 0; t < np; ++t) rmin = fmin(rmin, q[t][0]);
        const double e1 = fmin(rb, o->eps_bp);
        double th1 = 1.0;
        if (!(rmin >= e1)) th1 = fmin((rb - e1) / (rb - rmin), 1.0);
        for (int l = 1; l < o->nm; ++l) U(arr, c, 0, l) *= th1;
        /* step 2: internal energy E - |m|^2/(2 rho) of the density-limited state */
        double ub[NVAR];
        for (int v = 0; v < NVAR; ++v) ub[v] = U(arr, c, v, 0);
        const double eb = int_energy(ub);
        const double e2 = fmin(eb, o->eps_bp);
        limiter_values(o, arr, c, q);
        double emin = INFINITY;
        for (int t = 0; t < np; ++t) emin = fmin(emin, int_energy(q[t]));
        double th2 = 1.0;
        if (!(emin >= e2)) th2 = fmin((eb - e2) / (eb - emin), 1.0);
        for (int v = 0; v < NVAR; ++v)
            for (int l = 1; l < o->nm; ++l) U(arr, c, v, l) *= th2;
        if (th1 < 1.0 || th2 < 1.0) ++limited;
        if (!(rb > 0) || !(eb > 0)) ++bad;
    }
    o->n_limited += limited;
    return bad;
}

/* ----------------------------------------------------------------------- time stepping */

static void next_dt(Orc* o) {
    double dt = o->cssp * o->minck / o->alpha;
    const double rem = o->t_end - o->t;
    if (rem < dt) dt = rem;
    o->dt = dt;
    o->active = isinf(o->t_end) || rem > 1e-12 * fmax(1.0, fabs(o->t_end));
}

/* number of cells whose average leaves the admissible set (rho > 0, rho e > 0);
 * the OE filter and the limiter keep every average, so the pre-filter state has
 * the stage output's averages */
static int bad_averages(const Orc* o, const double* arr) {
    int bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : bad)
    for (int c = 0; c < o->nc; ++c) {
        double ub[NVAR];
        for (int v = 0; v < NVAR; ++v) ub[v] = U(arr, c, v, 0);
        if (!(ub[0] > 0) || !(int_energy(ub) > 0)) ++bad;
    }
    return bad;
}

/* eq. RKTime with the OE filter and the BP limiter after every stage (Sec. 4.5).
 * With the limiter on, a stage whose averages leave the admissible set sets
 * `skip`: the rest of the step does nothing and orc_step retries it. */
int orc_stage(Orc* o, int s) {
    const double a[3] = {0.0, 0.75, 1.0 / 3.0}, b[3] = {1.0, 0.25, 2.0 / 3.0};
    const size_t ns = (size_t)o->nc * NVAR * o->nm;
    if (s < 0 || s > 2) return -1;
    if (o->skip) return 0;
    const double* in = s == 0 ? o->u0 : o->u;
    const double alpha = max_wave_speed(o, in);
    if (s == 0) o->alpha = alpha;
    residual(o, in, alpha, o->L);
#pragma omp parallel for schedule(static)
    for (size_t i = 0; i < ns; ++i) o->w[i] = a[s] * o->u0[i] + b[s] * (in[i] + o->dt * o->L[i]);
    memcpy(o->pre, o->w, sizeof(double) * ns);
    if (o->bp_on && bad_averages(o, o->w)) {
        o->skip = 1;
        return 0;
    }
    if (o->oe_on) oe_filter(o, o->w, o->dt);
    if (o->bp_on && bp_limit(o, o->w)) o->err = -5;
    memcpy(o->u, o->w, sizeof(double) * ns);
    return o->err;
}

/* end of a step: u^{n+1} becomes u^n, t advances, alpha and Delta t of the new u^n */
int orc_finish_step(Orc* o) {
    memcpy(o->u0, o->u, sizeof(double) * (size_t)o->nc * NVAR * o->nm);
    o->t += o->dt;
    o->step += 1;
    o->alpha = max_wave_speed(o, o->u0);
    next_dt(o);
    return 0;
}

/* One step.  An attempt whose stage left the admissible set is discarded (u^n is
 * untouched) and the step is retried with half the time step, at most
 * max_restarts times; then the run stops with an error. */
int orc_step(Orc* o) {
    if (!o->active) return 1;
    for (;;) {
        o->skip = 0;
        for (int s = 0; s < 3 && !o->err && !o->skip; ++s) orc_stage(o, s);
        if (o->err) return o->err;
        if (!o->skip) break;
        o->skip = 0;
        if (++o->restarts_this_step > o->max_restarts) {
            o->err = -5;
            o->active = 0;
            return o->err;
        }
        o->dt *= 0.5;
        o->n_restarts++;
    }
    o->restarts_this_step = 0;
    return orc_finish_step(o);
}

int orc_set_max_restarts(Orc* o, int n) {
    o->max_restarts = n < 0 ? 0 : n;
    return 0;
}

int orc_run(Orc* o, double t_end, long max_steps, long* done) {
    long n = 0;
    if (t_end != o->t_end) {
        o->t_end = t_end;
        next_dt(o);
    }
    while (n < max_steps && o->active) {
        const int r = orc_step(o);
        if (r < 0) { if (done) *done = n; return r; }
        ++n;
    }
    if (done) *done = n;
    return 0;
}

/* ----------------------------------------------------------------------- initial data */

static void prim_to_cons(const Orc* o, const double* w, double* q) {
    q[0] = w[0];
    q[1] = w[0] * w[1];
    q[2] = w[0] * w[2];
    q[3] = w[3] / (o->gamma - 1.0) + 0.5 * w[0] * (w[1] * w[1] + w[2] * w[2]);
}

static void problem_state(const Orc* o, int kind, const double* P, double x, double y, double* q) {
    double w[4];
    if (kind == 0) {  /* isentropic vortex */
        const double xb = x - P[0], yb = y - P[1], r2 = xb * xb + yb * yb, g = o->gamma;
        const double amp = P[2] / (2.0 * M_PI) * exp(0.5 * (1.0 - r2));
        const double T = 1.0 - (g - 1.0) * P[2] * P[2] / (8.0 * g * M_PI * M_PI) * exp(1.0 - r2);
        w[0] = P[3] * pow(T, 1.0 / (g - 1.0));
        w[1] = P[4] - amp * yb;
        w[2] = P[5] + amp * xb;
        w[3] = pow(w[0], g) * (P[6] / pow(P[3], g));
    } else if (kind == 1) {  /* four quadrants */
        const int qd = (x >= P[0] ? 1 : 0) + (y >= P[1] ? 2 : 0);
        for (int i = 0; i < 4; ++i) w[i] = P[2 + 4 * qd + i];
    } else {  /* two states across a line */
        const int side = ((x - P[0]) * P[2] + (y - P[1]) * P[3]) < 0 ? 0 : 1;
        for (int i = 0; i < 4; ++i) w[i] = P[4 + 4 * side + i];
    }
    prim_to_cons(o, w, q);
}

int orc_init_modal(Orc* o, const double* u_soa) {
    const int nm = o->nm;
    for (int v = 0; v < NVAR; ++v)
        for (int l = 0; l < nm; ++l)
            for (int c = 0; c < o->nc; ++c) U(o->u0, c, v, l) = u_soa[((size_t)v * nm + l) * o->nc + c];
    return 0;
}

/* L2 projection with the 12-point rule, blast by cell averages */
int orc_init_problem(Orc* o, int kind, const double* P) {
    const int nm = o->nm;
    memset(o->u0, 0, sizeof(double) * (size_t)o->nc * NVAR * nm);
    if (kind == 2) {
        const int ov = (int)P[3];
        double at = 0;
        for (int c = 0; c < o->nc; ++c)
            if (local_vertex(o, c, ov) >= 0) at += o->area[c];
        for (int c = 0; c < o->nc; ++c) {
            const int hit = local_vertex(o, c, ov) >= 0;
            U(o->u0, c, 0, 0) = P[2];
            U(o->u0, c, 3, 0) = hit ? P[0] / at : P[1] / (o->gamma - 1.0);
        }
        return 0;
    }
#pragma omp parallel for schedule(static)
    for (int c = 0; c < o->nc; ++c) {
        const double* vc = o->vx + 6 * c;
        for (int m = 0; m < 12; ++m) {
            const double* b = TRI12_B[m];
            const double x = b[0] * vc[0] + b[1] * vc[2] + b[2] * vc[4];
            const double y = b[0] * vc[1] + b[1] * vc[3] + b[2] * vc[5];
            double q[NVAR], p[MAXM];
            problem_state(o, kind, P, x, y, q);
            basis(b[1], b[2], p);
            for (int v = 0; v < NVAR; ++v)
                for (int l = 0; l < nm; ++l) U(o->u0, c, v, l) += o->area[c] * TRI12_W[m] * q[v] * p[l];
        }
        for (int v = 0; v < NVAR; ++v)
            for (int l = 0; l < nm; ++l) U(o->u0, c, v, l) /= o->mass[(size_t)c * nm + l];
    }
    return 0;
}

/* after initial data: BP limiter (no OE), then alpha^0 and Delta t^0 */
int orc_start(Orc* o) {
    o->t = 0;
    o->step = 0;
    o->err = 0;
    o->n_limited = 0;
    o->skip = 0;
    o->restarts_this_step = 0;
    o->n_restarts = 0;
    o->t_end = INFINITY;
    if (o->bp_on && bp_limit(o, o->u0)) o->err = -5;
    memcpy(o->u, o->u0, sizeof(double) * (size_t)o->nc * NVAR * o->nm);
    o->alpha = max_wave_speed(o, o->u0);
    next_dt(o);
    return o->err;
}

/* ----------------------------------------------------------------------- accessors */

static void to_soa(const Orc* o, const double* arr, double* out) {
    const int nm = o->nm;
    for (int v = 0; v < NVAR; ++v)
        for (int l = 0; l < nm; ++l)
            for (int c = 0; c < o->nc; ++c) out[((size_t)v * nm + l) * o->nc + c] = U(arr, c, v, l);
}
static void from_soa(const Orc* o, const double* in, double* arr) {
    const int nm = o->nm;
    for (int v = 0; v < NVAR; ++v)
        for (int l = 0; l < nm; ++l)
            for (int c = 0; c < o->nc; ++c) U(arr, c, v, l) = in[((size_t)v * nm + l) * o->nc + c];
}

/* which: 0 = u^n (step start), 1 = current stage output, 2 = last pre-OE state */
int orc_get_state(const Orc* o, int which, double* out) {
    to_soa(o, which == 0 ? o->u0 : which == 1 ? o->u : o->pre, out);
    return 0;
}

/* scalars: t, dt, alpha, step, active, err, n_limited, minck,
 *          ubar[4], nrm_rho, nrm_m1, nrm_m2, nrm_E, nrm_m, zero_rho, zero_E, zero_m,
 *          n_restarts */
int orc_get_scalars(const Orc* o, double* s) {
    s[0] = o->t; s[1] = o->dt; s[2] = o->alpha; s[3] = (double)o->step; s[4] = o->active;
    s[5] = o->err; s[6] = (double)o->n_limited; s[7] = o->minck;
    for (int v = 0; v < 4; ++v) s[8 + v] = o->ubar[v];
    for (int v = 0; v < 4; ++v) s[12 + v] = o->nrm_v[v];
    s[16] = o->nrm_m; s[17] = o->zero_v[0]; s[18] = o->zero_v[3]; s[19] = o->zero_m;
    s[20] = (double)o->n_restarts;
    return 0;
}

int orc_set_time(Orc* o, double t, double dt, double alpha, long step) {
    o->t = t; o->dt = dt; o->alpha = alpha; o->step = step;
    return 0;
}

/* building blocks on an arbitrary SoA state, for the pins */
int orc_apply_residual(Orc* o, const double* in, double alpha, double* out) {
    from_soa(o, in, o->w);
    residual(o, o->w, alpha, o->pre);
    to_soa(o, o->pre, out);
    return 0;
}
int orc_apply_oe(Orc* o, double* inout, double dt) {
    from_soa(o, inout, o->w);
    oe_filter(o, o->w, dt);
    to_soa(o, o->w, inout);
    return 0;
}
int orc_apply_limiter(Orc* o, double* inout) {
    from_soa(o, inout, o->w);
    const int bad = bp_limit(o, o->w);
    to_soa(o, o->w, inout);
    return bad;
}
double orc_alpha_of(Orc* o, const double* in) {
    from_soa(o, in, o->w);
    return max_wave_speed(o, o->w);
}
/* values of every variable at the limiter's node set of each cell: out[c][t][v] */
int orc_limiter_node_values(Orc* o, const double* in, double* out) {
    from_soa(o, in, o->w);
    const int npt = o->k == 1 ? 8 : 11;
    for (int c = 0; c < o->nc; ++c) {
        double q[12][NVAR];
        limiter_values(o, o->w, c, q);
        for (int t = 0; t < npt; ++t)
            for (int v = 0; v < NVAR; ++v) out[((size_t)c * npt + t) * NVAR + v] = q[t][v];
    }
    return npt;
}
int orc_mass(const Orc* o, double* out) {
    memcpy(out, o->mass, sizeof(double) * (size_t)o->nc * o->nm);
    return 0;
}
/* basis values, used by the pins to check the basis against exact integrals */
void orc_basis(double xi, double eta, double* p, double* dxi, double* deta) {
    basis(xi, eta, p);
    basis_d1(xi, eta, dxi, deta);
}
/* quadrature tables: which 0 = 3-pt, 1 = 6-pt, 2 = 12-pt, 3 = edge Q=2, 4 = edge Q=3 */
int orc_quadrature(int which, double* pts, double* w) {
    init_consts();
    if (which == 0) { for (int m = 0; m < 3; ++m) { for (int i = 0; i < 3; ++i) pts[3 * m + i] = TRI3_B[m][i]; w[m] = TRI3_W[m]; } return 3; }
    if (which == 1) { for (int m = 0; m < 6; ++m) { for (int i = 0; i < 3; ++i) pts[3 * m + i] = TRI6_B[m][i]; w[m] = TRI6_W[m]; } return 6; }
    if (which == 2) { for (int m = 0; m < 12; ++m) { for (int i = 0; i < 3; ++i) pts[3 * m + i] = TRI12_B[m][i]; w[m] = TRI12_W[m]; } return 12; }
    const int Q = which == 3 ? 2 : 3;
    for (int g = 0; g < Q; ++g) { pts[g] = GS[Q][g]; w[g] = GW[Q][g]; }
    return Q;
}

/* Threads of the cell loops (OpenMP; n <= 0: one per processor); returns the
 * number now in use, 1 without OpenMP. */
int orc_set_threads(int n) {
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : omp_get_num_procs());
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}
