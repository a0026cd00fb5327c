/*
 * pf_oracle.c -- plain FP64 CPU oracle for batched Newton-Raphson AC power flow.
 *
 * TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.  Only the test suite, the smoke check
 * and the CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the GPU path.
 *
 * What it computes (Wang, Wende-von Berg, Braun, "Fast parallel Newton-Raphson power
 * flow solver for large number of system calculations with CPU and GPU"):
 *   * nodal power S = V o conj(Ybus V)                                    (Sec. 3, Eq. 1)
 *   * mismatch F = [Re(S - S_sp) at pv,pq buses ; Im(S - S_sp) at pq buses], with the
 *     calculated power minus the specified one, as the NPM kernel initialises the
 *     mismatch with minus the specified injection                         (Sec. 3.1.1, Alg. 1)
 *   * the NR loop: mismatch -> Jacobian -> linear solve -> voltage update, stopping when
 *     the largest mismatch drops below the tolerance or at the iteration limit (Sec. 3)
 *   * the Jacobian d{P,Q}/d{angle V, |V|} restricted to the unknowns
 *     x = [angle V at pv,pq ; |V| at pq] and equations [dP at pv,pq ; dQ at pq]
 *                                                                         (Sec. 3.1.2, Eq. 2)
 *   * the linear solve by a fill-reducing pre-order and a left-looking Gilbert-Peierls
 *     LU with partial pivoting, then forward/backward substitution        (Sec. 4.1, Eq. 3;
 *                                                                          Sec. 4.2, Alg. 2)
 *
 * Readings of points the paper leaves open (see the design notes of the repository):
 *   * update sign: x solves J x = F with F = calculated - specified, so V <- V - x;
 *   * convergence: infinity norm of F, strictly below tol, tested before every update
 *     including the first; iters = number of updates performed;
 *   * |V| derivatives are the unscaled d/d|V| ("d{P,Q}/d{angle V, |V|}");
 *   * unknown/equation order: pv buses then pq buses, each ascending by bus index;
 *   * the pre-order is a plain minimum-degree ordering of the (structurally symmetric)
 *     Jacobian graph; pivoting is threshold partial pivoting (threshold 0.1) that prefers
 *     the diagonal of the pre-ordered matrix, re-done at every iteration.
 *
 * Everything here is deliberately straightforward: dense scatter vectors, explicit
 * depth-first reach, no blocking or vectorisation.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define BUS_PQ 1
#define BUS_PV 2
#define BUS_REF 3

enum { ST_CONVERGED = 0, ST_MAXITER = 1, ST_NONFINITE = 2, ST_SINGULAR = 3 };

/* ------------------------------------------------------------------ min-degree order */
/*
 * Plain minimum-degree ordering on an undirected graph given by a symmetric CSR pattern
 * (diagonal entries ignored).  The elimination graph is kept as a dense bitset; at each
 * step the uneliminated vertex of smallest current degree (ties: smallest index) is
 * eliminated and its neighbours are joined into a clique.
 */
static int min_degree_order(int N, const int *rp, const int *ci, int *order)
{
    size_t words = ((size_t)N + 63) / 64;
    uint64_t *adj = (uint64_t *)calloc((size_t)N * words, sizeof(uint64_t));
    int *deg = (int *)calloc((size_t)N, sizeof(int));
    char *gone = (char *)calloc((size_t)N, 1);
    int *nb = (int *)malloc(sizeof(int) * (size_t)(N > 0 ? N : 1));
    if (!adj || !deg || !gone || !nb) {
        free(adj); free(deg); free(gone); free(nb);
        return -1;
    }
#define ADJ(a, b) (adj[(size_t)(a) * words + ((size_t)(b) >> 6)] >> ((b) & 63) & 1ULL)
#define SETADJ(a, b) (adj[(size_t)(a) * words + ((size_t)(b) >> 6)] |= 1ULL << ((b) & 63))
#define CLRADJ(a, b) (adj[(size_t)(a) * words + ((size_t)(b) >> 6)] &= ~(1ULL << ((b) & 63)))
    for (int i = 0; i < N; i++)
        for (int p = rp[i]; p < rp[i + 1]; p++) {
            int j = ci[p];
            if (j == i) continue;
            if (!ADJ(i, j)) { SETADJ(i, j); deg[i]++; }
            if (!ADJ(j, i)) { SETADJ(j, i); deg[j]++; }
        }
    for (int step = 0; step < N; step++) {
        int v = -1;
        for (int i = 0; i < N; i++)
            if (!gone[i] && (v < 0 || deg[i] < deg[v])) v = i;
        order[step] = v;
        int cnt = 0;
        for (int u = 0; u < N; u++)
            if (!gone[u] && u != v && ADJ(v, u)) nb[cnt++] = u;
        for (int a = 0; a < cnt; a++)
            for (int b = a + 1; b < cnt; b++) {
                int x = nb[a], y = nb[b];
                if (!ADJ(x, y)) {
                    SETADJ(x, y); SETADJ(y, x);
                    deg[x]++; deg[y]++;
                }
            }
        for (int a = 0; a < cnt; a++) {
            CLRADJ(nb[a], v);
            deg[nb[a]]--;
        }
        gone[v] = 1;
    }
#undef ADJ
#undef SETADJ
#undef CLRADJ
    free(adj); free(deg); free(gone); free(nb);
    return 0;
}

/* ------------------------------------------------------------------ sparse LU (G-P) */
typedef struct {
    int N;
    /* L: unit lower, column k holds (original row index, value) with the diagonal omitted */
    int *lp, *li; double *lx; int lcap;
    /* U: column k holds (pivot step j < k, value); diagonal in ud[k] */
    int *up, *ui; double *ux; int ucap;
    double *ud;
    int *pinv;    /* original row -> pivot step, -1 while not pivotal */
    int *prow;    /* pivot step -> original row */
    /* scratch */
    double *x; int *mark; int *stack; int *pstack; int *topo; int *pat;
} lu_t;

static void lu_free(lu_t *f)
{
    free(f->lp); free(f->li); free(f->lx);
    free(f->up); free(f->ui); free(f->ux); free(f->ud);
    free(f->pinv); free(f->prow);
    free(f->x); free(f->mark); free(f->stack); free(f->pstack); free(f->topo); free(f->pat);
    memset(f, 0, sizeof(*f));
}

static int lu_init(lu_t *f, int N, int cap)
{
    memset(f, 0, sizeof(*f));
    f->N = N;
    if (cap < 16) cap = 16;
    f->lcap = f->ucap = cap;
    size_t n1 = (size_t)N + 1, nn = (size_t)(N > 0 ? N : 1);
    f->lp = malloc(sizeof(int) * n1); f->li = malloc(sizeof(int) * (size_t)cap);
    f->lx = malloc(sizeof(double) * (size_t)cap);
    f->up = malloc(sizeof(int) * n1); f->ui = malloc(sizeof(int) * (size_t)cap);
    f->ux = malloc(sizeof(double) * (size_t)cap);
    f->ud = malloc(sizeof(double) * nn);
    f->pinv = malloc(sizeof(int) * nn); f->prow = malloc(sizeof(int) * nn);
    f->x = calloc(nn, sizeof(double)); f->mark = calloc(nn, sizeof(int));
    f->stack = malloc(sizeof(int) * nn); f->pstack = malloc(sizeof(int) * nn);
    f->topo = malloc(sizeof(int) * nn); f->pat = malloc(sizeof(int) * nn);
    if (!f->lp || !f->li || !f->lx || !f->up || !f->ui || !f->ux || !f->ud || !f->pinv ||
        !f->prow || !f->x || !f->mark || !f->stack || !f->pstack || !f->topo || !f->pat) {
        lu_free(f);
        return -1;
    }
    return 0;
}

static int grow(int **i, double **v, int *cap, int need)
{
    if (need <= *cap) return 0;
    int nc = *cap;
    while (nc < need) nc *= 2;
    int *ni = realloc(*i, sizeof(int) * (size_t)nc);
    if (!ni) return -1;
    *i = ni;
    double *nv = realloc(*v, sizeof(double) * (size_t)nc);
    if (!nv) return -1;
    *v = nv;
    *cap = nc;
    return 0;
}

/*
 * Left-looking LU with partial pivoting of the CSC matrix A (cp, ri, av), columns taken
 * in the order q[k] (Sec. 4.2, Alg. 2: copy the column into a working space, apply the
 * sparse VMAD of every earlier column it depends on, then split into U and L).
 * Pivot choice: the preferred row q[k] (the diagonal of the symmetrically pre-ordered
 * matrix) if |x| there is at least 0.1 of the column maximum, else the maximum.
 * Returns 0, or ST_SINGULAR if a column has no usable pivot.
 */
static int lu_factor(lu_t *f, const int *cp, const int *ri, const double *av, const int *q)
{
    int N = f->N;
    for (int i = 0; i < N; i++) { f->pinv[i] = -1; f->mark[i] = -1; }
    f->lp[0] = 0; f->up[0] = 0;
    for (int k = 0; k < N; k++) {
        int col = q[k];
        /* reach of column col in the graph of L, in topological order (depth-first) */
        int ntopo = 0, npat = 0;
        for (int p = cp[col]; p < cp[col + 1]; p++) {
            int r0 = ri[p];
            if (f->mark[r0] == k) continue;
            int sp = 0;
            f->stack[0] = r0; f->pstack[0] = -1; f->mark[r0] = k;
            while (sp >= 0) {
                int r = f->stack[sp];
                int j = f->pinv[r];
                if (f->pstack[sp] < 0) f->pstack[sp] = (j >= 0) ? f->lp[j] : 0;
                int pushed = 0;
                if (j >= 0) {
                    int end = f->lp[j + 1];
                    while (f->pstack[sp] < end) {
                        int c = f->li[f->pstack[sp]++];
                        if (f->mark[c] != k) {
                            f->mark[c] = k;
                            sp++;
                            f->stack[sp] = c; f->pstack[sp] = -1;
                            pushed = 1;
                            break;
                        }
                    }
                }
                if (!pushed) { f->topo[ntopo++] = r; sp--; }
            }
        }
        /* topo holds a post-order: process it reversed */
        for (int p = cp[col]; p < cp[col + 1]; p++) f->x[ri[p]] = av[p];
        for (int t = ntopo - 1; t >= 0; t--) {
            int r = f->topo[t];
            f->pat[npat++] = r;
            int j = f->pinv[r];
            if (j < 0) continue;
            double xr = f->x[r];
            for (int p = f->lp[j]; p < f->lp[j + 1]; p++) f->x[f->li[p]] -= f->lx[p] * xr;
        }
        /* split: U part (pivotal rows), pivot search among the others */
        int unz = f->up[k], lnz = f->lp[k];
        if (grow(&f->ui, &f->ux, &f->ucap, unz + npat) || grow(&f->li, &f->lx, &f->lcap, lnz + npat))
            return -1;
        double amax = -1.0; int ipiv = -1;
        for (int t = 0; t < npat; t++) {
            int r = f->pat[t];
            if (f->pinv[r] >= 0) {
                f->ui[unz] = f->pinv[r]; f->ux[unz] = f->x[r]; unz++;
            } else {
                double a = fabs(f->x[r]);
                if (a > amax) { amax = a; ipiv = r; }
            }
        }
        int pref = q[k];
        if (f->pinv[pref] < 0 && f->mark[pref] == k && fabs(f->x[pref]) >= 0.1 * amax) ipiv = pref;
        if (ipiv < 0 || !(amax > 0.0) || !isfinite(f->x[ipiv])) {
            for (int t = 0; t < npat; t++) f->x[f->pat[t]] = 0.0;
            return ST_SINGULAR;
        }
        double piv = f->x[ipiv];
        f->ud[k] = piv;
        f->pinv[ipiv] = k; f->prow[k] = ipiv;
        for (int t = 0; t < npat; t++) {
            int r = f->pat[t];
            if (f->pinv[r] < 0) {
                f->li[lnz] = r; f->lx[lnz] = f->x[r] / piv; lnz++;
            }
            f->x[r] = 0.0;
        }
        f->up[k + 1] = unz; f->lp[k + 1] = lnz;
    }
    return 0;
}

/* Solve A x = b with the factors of lu_factor (P A Q = L U): forward, backward, permute. */
static void lu_solve(lu_t *f, const int *q, const double *b, double *xout)
{
    int N = f->N;
    double *w = f->x;   /* indexed by pivot step */
    for (int i = 0; i < N; i++) w[f->pinv[i]] = b[i];
    for (int k = 0; k < N; k++) {
        double yk = w[k];
        for (int p = f->lp[k]; p < f->lp[k + 1]; p++) w[f->pinv[f->li[p]]] -= f->lx[p] * yk;
    }
    for (int k = N - 1; k >= 0; k--) {
        double zk = w[k] / f->ud[k];
        w[k] = zk;
        for (int p = f->up[k]; p < f->up[k + 1]; p++) w[f->ui[p]] -= f->ux[p] * zk;
    }
    for (int k = 0; k < N; k++) xout[q[k]] = w[k];
    for (int k = 0; k < N; k++) w[k] = 0.0;
}

/* ------------------------------------------------------------------ power-flow system */
typedef struct {
    int n, nnzy;
    int *rp, *ci;
    double *g, *b;          /* Ybus real and imaginary parts */
    signed char *bt;
    int npv, npq, npvpq, N;
    int *th;                /* bus -> index of its angle unknown, or -1 */
    int *vm;                /* bus -> index of its |V| unknown, or -1 */
    int *ubus;              /* unknown/equation index -> bus */
    /* Jacobian pattern, CSR by equation, and its CSC copy by unknown */
    int nnzj;
    int *jrp, *jci;         /* CSR */
    int *jy;                /* CSR entry -> Ybus entry */
    int *ccp, *cri, *cmap;  /* CSC pattern and CSR->CSC position map */
    int *order;             /* minimum-degree order of the unknowns */
} pfsys_t;

void oracle_destroy(void *h)
{
    pfsys_t *s = (pfsys_t *)h;
    if (!s) return;
    free(s->rp); free(s->ci); free(s->g); free(s->b); free(s->bt);
    free(s->th); free(s->vm); free(s->ubus);
    free(s->jrp); free(s->jci); free(s->jy); free(s->ccp); free(s->cri); free(s->cmap);
    free(s->order);
    free(s);
}

/*
 * Build the system: bus classification, unknown numbering, Jacobian pattern (rows and
 * columns follow the unknown order) and its minimum-degree order.  y holds the Ybus
 * values as interleaved (re, im) pairs.  Returns NULL on invalid input.
 */
void *oracle_create(int n, const int *rp, const int *ci, const double *y, const signed char *bt)
{
    if (n <= 0 || !rp || !ci || !y || !bt) return NULL;
    pfsys_t *s = (pfsys_t *)calloc(1, sizeof(pfsys_t));
    if (!s) return NULL;
    int nnz = rp[n];
    s->n = n; s->nnzy = nnz;
    s->rp = malloc(sizeof(int) * (size_t)(n + 1)); s->ci = malloc(sizeof(int) * (size_t)nnz);
    s->g = malloc(sizeof(double) * (size_t)nnz); s->b = malloc(sizeof(double) * (size_t)nnz);
    s->bt = malloc((size_t)n);
    s->th = malloc(sizeof(int) * (size_t)n); s->vm = malloc(sizeof(int) * (size_t)n);
    s->ubus = malloc(sizeof(int) * (size_t)(2 * n));
    if (!s->rp || !s->ci || !s->g || !s->b || !s->bt || !s->th || !s->vm || !s->ubus) goto fail;
    memcpy(s->rp, rp, sizeof(int) * (size_t)(n + 1));
    memcpy(s->ci, ci, sizeof(int) * (size_t)nnz);
    memcpy(s->bt, bt, (size_t)n);
    for (int p = 0; p < nnz; p++) { s->g[p] = y[2 * p]; s->b[p] = y[2 * p + 1]; }
    int nref = 0;
    for (int i = 0; i < n; i++) {
        if (bt[i] == BUS_PV) s->npv++;
        else if (bt[i] == BUS_PQ) s->npq++;
        else if (bt[i] == BUS_REF) nref++;
        else goto fail;
    }
    if (nref != 1) goto fail;
    s->npvpq = s->npv + s->npq;
    s->N = s->npvpq + s->npq;
    int u = 0;
    for (int i = 0; i < n; i++) { s->th[i] = -1; s->vm[i] = -1; }
    for (int i = 0; i < n; i++) if (bt[i] == BUS_PV) { s->th[i] = u; s->ubus[u++] = i; }
    for (int i = 0; i < n; i++) if (bt[i] == BUS_PQ) { s->th[i] = u; s->ubus[u++] = i; }
    for (int i = 0; i < n; i++) if (bt[i] == BUS_PQ) { s->vm[i] = u; s->ubus[u++] = i; }
    int N = s->N;
    /* Jacobian pattern: equation row r of bus i couples with every unknown of every bus
       k in row i of Ybus.  Columns are emitted in ascending unknown index. */
    s->jrp = malloc(sizeof(int) * (size_t)(N + 1));
    if (!s->jrp) goto fail;
    int cap = 4 * nnz + 4;
    s->jci = malloc(sizeof(int) * (size_t)cap); s->jy = malloc(sizeof(int) * (size_t)cap);
    int *tmpc = malloc(sizeof(int) * (size_t)(2 * n + 2)), *tmpy = malloc(sizeof(int) * (size_t)(2 * n + 2));
    if (!s->jci || !s->jy || !tmpc || !tmpy) { free(tmpc); free(tmpy); goto fail; }
    int nz = 0;
    s->jrp[0] = 0;
    for (int r = 0; r < N; r++) {
        int i = s->ubus[r];
        int cnt = 0;
        for (int p = rp[i]; p < rp[i + 1]; p++) {
            int k = ci[p];
            if (s->th[k] >= 0) { tmpc[cnt] = s->th[k]; tmpy[cnt] = p; cnt++; }
            if (s->vm[k] >= 0) { tmpc[cnt] = s->vm[k]; tmpy[cnt] = p; cnt++; }
        }
        /* insertion sort by column */
        for (int a = 1; a < cnt; a++) {
            int c = tmpc[a], yy = tmpy[a], b2 = a - 1;
            while (b2 >= 0 && tmpc[b2] > c) { tmpc[b2 + 1] = tmpc[b2]; tmpy[b2 + 1] = tmpy[b2]; b2--; }
            tmpc[b2 + 1] = c; tmpy[b2 + 1] = yy;
        }
        for (int a = 0; a < cnt; a++) { s->jci[nz] = tmpc[a]; s->jy[nz] = tmpy[a]; nz++; }
        s->jrp[r + 1] = nz;
    }
    free(tmpc); free(tmpy);
    s->nnzj = nz;
    /* CSC copy */
    s->ccp = calloc((size_t)(N + 1), sizeof(int));
    s->cri = malloc(sizeof(int) * (size_t)(nz > 0 ? nz : 1));
    s->cmap = malloc(sizeof(int) * (size_t)(nz > 0 ? nz : 1));
    s->order = malloc(sizeof(int) * (size_t)(N > 0 ? N : 1));
    if (!s->ccp || !s->cri || !s->cmap || !s->order) goto fail;
    for (int p = 0; p < nz; p++) s->ccp[s->jci[p] + 1]++;
    for (int c = 0; c < N; c++) s->ccp[c + 1] += s->ccp[c];
    int *fillp = malloc(sizeof(int) * (size_t)(N > 0 ? N : 1));
    if (!fillp) goto fail;
    for (int c = 0; c < N; c++) fillp[c] = s->ccp[c];
    for (int r = 0; r < N; r++)
        for (int p = s->jrp[r]; p < s->jrp[r + 1]; p++) {
            int c = s->jci[p];
            s->cri[fillp[c]] = r;
            s->cmap[p] = fillp[c]++;
        }
    free(fillp);
    if (min_degree_order(N, s->jrp, s->jci, s->order)) goto fail;
    return s;
fail:
    oracle_destroy(s);
    return NULL;
}

int oracle_dims(void *h, int *out)
{
    pfsys_t *s = (pfsys_t *)h;
    if (!s || !out) return -1;
    out[0] = s->n; out[1] = s->npv; out[2] = s->npq; out[3] = s->N; out[4] = s->nnzj;
    return 0;
}

int oracle_order(void *h, int *perm)
{
    pfsys_t *s = (pfsys_t *)h;
    if (!s || !perm) return -1;
    memcpy(perm, s->order, sizeof(int) * (size_t)s->N);
    return 0;
}

int oracle_jacobian_pattern(void *h, int *jrp, int *jci)
{
    pfsys_t *s = (pfsys_t *)h;
    if (!s) return -1;
    memcpy(jrp, s->jrp, sizeof(int) * (size_t)(s->N + 1));
    memcpy(jci, s->jci, sizeof(int) * (size_t)s->nnzj);
    return 0;
}

/* Complex current injections I = Ybus V and polar-to-rectangular V (Eq. 1). */
static void currents(const pfsys_t *s, const double *vm, const double *va,
                     double *vr, double *vi, double *ir, double *ii)
{
    for (int i = 0; i < s->n; i++) { vr[i] = vm[i] * cos(va[i]); vi[i] = vm[i] * sin(va[i]); }
    for (int i = 0; i < s->n; i++) {
        double ar = 0.0, ai = 0.0;
        for (int p = s->rp[i]; p < s->rp[i + 1]; p++) {
            int k = s->ci[p];
            ar += s->g[p] * vr[k] - s->b[p] * vi[k];
            ai += s->g[p] * vi[k] + s->b[p] * vr[k];
        }
        ir[i] = ar; ii[i] = ai;
    }
}

/* F = [Re(S - Ssp)]_{pv,pq} ++ [Im(S - Ssp)]_{pq},  S = V conj(I); returns max |F| (or NaN). */
static double mismatch(const pfsys_t *s, const double *vr, const double *vi, const double *ir,
                       const double *ii, const double *sp, const double *sq, double *F)
{
    double nf = 0.0;
    int finite = 1;
    for (int u = 0; u < s->N; u++) {
        int i = s->ubus[u];
        double pr = vr[i] * ir[i] + vi[i] * ii[i];    /* Re(V conj I) */
        double qr = vi[i] * ir[i] - vr[i] * ii[i];    /* Im(V conj I) */
        double f = (u < s->npvpq) ? pr - sp[i] : qr - sq[i];
        F[u] = f;
        if (!isfinite(f)) finite = 0;
        else if (fabs(f) > nf) nf = fabs(f);
    }
    return finite ? nf : NAN;
}

/*
 * Jacobian values in the CSR pattern (Sec. 3.1.2).  With V_i = |V_i| e^{j th_i},
 * I = Y V and S_i = V_i conj(I_i):
 *   dS_i/dth_k   = -j V_i conj(Y_ik V_k)                      (k != i)
 *   dS_i/dth_i   =  j S_i - j |V_i|^2 conj(Y_ii)
 *   dS_i/d|V_k|  =  V_i conj(Y_ik V_k) / |V_k|                (k != i)
 *   dS_i/d|V_i|  =  S_i / |V_i| + |V_i| conj(Y_ii)
 * P equations take the real part, Q equations the imaginary part.
 */
static void jacobian(const pfsys_t *s, const double *vm, const double *vr, const double *vi,
                     const double *ir, const double *ii, double *J)
{
    for (int r = 0; r < s->N; r++) {
        int i = s->ubus[r];
        int isq = (r >= s->npvpq);
        double sr = vr[i] * ir[i] + vi[i] * ii[i];
        double si = vi[i] * ir[i] - vr[i] * ii[i];
        for (int p = s->jrp[r]; p < s->jrp[r + 1]; p++) {
            int c = s->jci[p];
            int k = s->ubus[c];
            int wrt_vm = (c >= s->npvpq);
            int q = s->jy[p];
            double gr = s->g[q], gi = s->b[q];
            double dr, di;   /* the complex derivative dS_i/d(unknown c) */
            if (k != i) {
                /* w = V_i conj(Y_ik V_k) */
                double yvr = gr * vr[k] - gi * vi[k], yvi = gr * vi[k] + gi * vr[k];
                double wr = vr[i] * yvr + vi[i] * yvi;
                double wi = vi[i] * yvr - vr[i] * yvi;
                if (!wrt_vm) { dr = wi; di = -wr; }          /* -j w */
                else { dr = wr / vm[k]; di = wi / vm[k]; }
            } else {
                double m2 = vm[i] * vm[i];
                if (!wrt_vm) { dr = -si - m2 * gi; di = sr - m2 * gr; }   /* j S - j m2 conj(Y) */
                else { dr = sr / vm[i] + vm[i] * gr; di = si / vm[i] - vm[i] * gi; }
            }
            J[p] = isq ? di : dr;
        }
    }
}

/* ---------------------------------------------------------------- exported building blocks */
/* sbus, v: interleaved [n][2]; F: [N].  Returns 0. */
int oracle_mismatch(void *h, const double *sbus, const double *v, double *F, double *normF)
{
    pfsys_t *s = (pfsys_t *)h;
    int n = s->n;
    double *w = malloc(sizeof(double) * (size_t)n * 8);
    if (!w) return -1;
    double *vm = w, *va = w + n, *vr = w + 2 * n, *vi = w + 3 * n, *ir = w + 4 * n, *ii = w + 5 * n;
    double *sp = w + 6 * n, *sq = w + 7 * n;
    for (int i = 0; i < n; i++) { vm[i] = v[2 * i]; va[i] = v[2 * i + 1]; sp[i] = sbus[2 * i]; sq[i] = sbus[2 * i + 1]; }
    currents(s, vm, va, vr, vi, ir, ii);
    double nf = mismatch(s, vr, vi, ir, ii, sp, sq, F);
    if (normF) *normF = nf;
    free(w);
    return 0;
}

/* Jacobian values at V in the CSR pattern of oracle_jacobian_pattern. */
int oracle_jacobian(void *h, const double *v, double *J)
{
    pfsys_t *s = (pfsys_t *)h;
    int n = s->n;
    double *w = malloc(sizeof(double) * (size_t)n * 6);
    if (!w) return -1;
    double *vm = w, *va = w + n, *vr = w + 2 * n, *vi = w + 3 * n, *ir = w + 4 * n, *ii = w + 5 * n;
    for (int i = 0; i < n; i++) { vm[i] = v[2 * i]; va[i] = v[2 * i + 1]; }
    currents(s, vm, va, vr, vi, ir, ii);
    jacobian(s, vm, vr, vi, ir, ii, J);
    free(w);
    return 0;
}

/* Solve J x = rhs for Jacobian values given in the CSR pattern (LU with pivoting). */
int oracle_jacobian_solve(void *h, const double *J, const double *rhs, double *x)
{
    pfsys_t *s = (pfsys_t *)h;
    int N = s->N;
    double *av = malloc(sizeof(double) * (size_t)(s->nnzj > 0 ? s->nnzj : 1));
    lu_t f;
    if (!av || lu_init(&f, N, 4 * s->nnzj)) { free(av); return -1; }
    for (int p = 0; p < s->nnzj; p++) av[s->cmap[p]] = J[p];
    int rc = lu_factor(&f, s->ccp, s->cri, av, s->order);
    if (rc == 0) lu_solve(&f, s->order, rhs, x);
    lu_free(&f);
    free(av);
    return rc;
}

/*
 * General sparse solve A x = b for a square CSR matrix (test entry point): the same
 * minimum-degree pre-order (on the pattern of A + A^T) and pivoting LU.
 */
int oracle_sparse_solve(int N, const int *rp, const int *ci, const double *val,
                        const double *b, double *x)
{
    if (N <= 0) return 0;
    int nz = rp[N];
    /* CSC of A */
    int *cp = calloc((size_t)N + 1, sizeof(int));
    int *ri = malloc(sizeof(int) * (size_t)(nz > 0 ? nz : 1));
    double *av = malloc(sizeof(double) * (size_t)(nz > 0 ? nz : 1));
    int *fp = malloc(sizeof(int) * (size_t)N);
    /* symmetric pattern A + A^T as CSR (may contain duplicates, harmless for ordering) */
    int *sp2 = calloc((size_t)N + 1, sizeof(int));
    int *sc2 = malloc(sizeof(int) * (size_t)(2 * nz + 1));
    int *order = malloc(sizeof(int) * (size_t)N);
    int rc = -1;
    if (!cp || !ri || !av || !fp || !sp2 || !sc2 || !order) goto out;
    for (int p = 0; p < nz; p++) cp[ci[p] + 1]++;
    for (int c = 0; c < N; c++) cp[c + 1] += cp[c];
    for (int c = 0; c < N; c++) fp[c] = cp[c];
    for (int r = 0; r < N; r++)
        for (int p = rp[r]; p < rp[r + 1]; p++) { int c = ci[p]; ri[fp[c]] = r; av[fp[c]] = val[p]; fp[c]++; }
    for (int r = 0; r < N; r++)
        for (int p = rp[r]; p < rp[r + 1]; p++) { sp2[r + 1]++; sp2[ci[p] + 1]++; }
    for (int r = 0; r < N; r++) sp2[r + 1] += sp2[r];
    for (int r = 0; r < N; r++) fp[r] = sp2[r];
    for (int r = 0; r < N; r++)
        for (int p = rp[r]; p < rp[r + 1]; p++) { sc2[fp[r]++] = ci[p]; sc2[fp[ci[p]]++] = r; }
    if (min_degree_order(N, sp2, sc2, order)) goto out;
    lu_t f;
    if (lu_init(&f, N, 4 * nz)) goto out;
    rc = lu_factor(&f, cp, ri, av, order);
    if (rc == 0) lu_solve(&f, order, b, x);
    lu_free(&f);
out:
    free(cp); free(ri); free(av); free(fp); free(sp2); free(sc2); free(order);
    return rc;
}

/* Branch flows of pi-model branches (from the branch list, independent of Ybus):
   S_f = V_f conj(I_f), I_f = (y_s + j b/2) V_f - y_s V_t;  S_t likewise. */
int oracle_branch_flows(int n, int m, const int *fb, const int *tb, const double *r,
                        const double *xb, const double *bb, const double *v, double *sf, double *st)
{
    (void)n;
    for (int e = 0; e < m; e++) {
        int f = fb[e], t = tb[e];
        double d = r[e] * r[e] + xb[e] * xb[e];
        double ysr = r[e] / d, ysi = -xb[e] / d;
        double vfr = v[2 * f] * cos(v[2 * f + 1]), vfi = v[2 * f] * sin(v[2 * f + 1]);
        double vtr = v[2 * t] * cos(v[2 * t + 1]), vti = v[2 * t] * sin(v[2 * t + 1]);
        double hb = 0.5 * bb[e];
        /* I_f = ys (Vf - Vt) + j hb Vf */
        double dr = vfr - vtr, di = vfi - vti;
        double ifr = ysr * dr - ysi * di - hb * vfi;
        double ifi = ysr * di + ysi * dr + hb * vfr;
        double itr = -(ysr * dr - ysi * di) - hb * vti;
        double iti = -(ysr * di + ysi * dr) + hb * vtr;
        sf[2 * e] = vfr * ifr + vfi * ifi; sf[2 * e + 1] = vfi * ifr - vfr * ifi;
        st[2 * e] = vtr * itr + vti * iti; st[2 * e + 1] = vti * itr - vtr * iti;
    }
    return 0;
}

/* ------------------------------------------------------------------ batched NR driver */
typedef struct {
    pfsys_t *s;
    int batch; const double *sbus; const double *v0;
    double tol; int max_iter;
    double *v_out; int *iters; unsigned char *conv; signed char *status; double *hist;
    volatile int next;
    pthread_mutex_t lock;
} job_t;

/* One instance of the NR loop (Sec. 3): mismatch and convergence test, Jacobian, solve,
   update; repeated until converged, non-finite, singular or at max_iter. */
static void solve_one(pfsys_t *s, lu_t *f, double *w, double *av, int b, job_t *jb)
{
    int n = s->n, N = s->N;
    double *vm = w, *va = w + n, *vr = w + 2 * n, *vi = w + 3 * n, *ir = w + 4 * n, *ii = w + 5 * n;
    double *sp = w + 6 * n, *sq = w + 7 * n;
    double *F = w + 8 * n, *dx = w + 8 * n + N, *J = w + 8 * n + 2 * N;
    const double *sb = jb->sbus + (size_t)b * n * 2, *v0 = jb->v0 + (size_t)b * n * 2;
    double *hist = jb->hist ? jb->hist + (size_t)b * (jb->max_iter + 1) : NULL;
    for (int i = 0; i < n; i++) { vm[i] = v0[2 * i]; va[i] = v0[2 * i + 1]; sp[i] = sb[2 * i]; sq[i] = sb[2 * i + 1]; }
    if (hist) for (int k = 0; k <= jb->max_iter; k++) hist[k] = NAN;
    int k = 0, st = ST_MAXITER;
    for (;;) {
        currents(s, vm, va, vr, vi, ir, ii);
        double nf = mismatch(s, vr, vi, ir, ii, sp, sq, F);
        if (hist) hist[k] = nf;
        if (!isfinite(nf)) { st = ST_NONFINITE; break; }
        if (nf < jb->tol) { st = ST_CONVERGED; break; }
        if (k >= jb->max_iter) { st = ST_MAXITER; break; }
        jacobian(s, vm, vr, vi, ir, ii, J);
        for (int p = 0; p < s->nnzj; p++) av[s->cmap[p]] = J[p];
        if (lu_factor(f, s->ccp, s->cri, av, s->order)) { st = ST_SINGULAR; break; }
        lu_solve(f, s->order, F, dx);
        for (int u = 0; u < s->npvpq; u++) va[s->ubus[u]] -= dx[u];
        for (int u = s->npvpq; u < N; u++) vm[s->ubus[u]] -= dx[u];
        k++;
    }
    double *vo = jb->v_out + (size_t)b * n * 2;
    for (int i = 0; i < n; i++) { vo[2 * i] = vm[i]; vo[2 * i + 1] = va[i]; }
    jb->iters[b] = k;
    jb->conv[b] = (st == ST_CONVERGED);
    if (jb->status) jb->status[b] = (signed char)st;
}

static void *worker(void *arg)
{
    job_t *jb = (job_t *)arg;
    pfsys_t *s = jb->s;
    int n = s->n, N = s->N;
    double *w = malloc(sizeof(double) * ((size_t)8 * n + 2 * (size_t)N + (size_t)s->nnzj + 1));
    double *av = malloc(sizeof(double) * ((size_t)s->nnzj + 1));
    lu_t f;
    int ok = (w && av && lu_init(&f, N, 4 * s->nnzj) == 0);
    for (;;) {
        pthread_mutex_lock(&jb->lock);
        int b = jb->next++;
        pthread_mutex_unlock(&jb->lock);
        if (b >= jb->batch) break;
        if (!ok) { jb->iters[b] = 0; jb->conv[b] = 0; if (jb->status) jb->status[b] = -1; continue; }
        solve_one(s, &f, w, av, b, jb);
    }
    if (ok) lu_free(&f);
    free(w); free(av);
    return NULL;
}

/*
 * Solve `batch` independent power flows that share the Ybus of h.
 *   sbus, v0, v_out: [batch][n][2] = (P, Q) / (|V|, theta) interleaved doubles
 *   iters [batch], conv [batch], status [batch] (may be NULL), hist [batch][max_iter+1]
 *   (may be NULL) receives max|F| at every mismatch evaluation (NaN after the stop).
 * nthreads workers take instances one at a time.  Returns 0.
 */
int oracle_nr(void *h, int batch, const double *sbus, const double *v0, double tol, int max_iter,
              int nthreads, double *v_out, int *iters, unsigned char *conv, signed char *status,
              double *hist)
{
    job_t jb;
    memset(&jb, 0, sizeof(jb));
    jb.s = (pfsys_t *)h; jb.batch = batch; jb.sbus = sbus; jb.v0 = v0; jb.tol = tol;
    jb.max_iter = max_iter; jb.v_out = v_out; jb.iters = iters; jb.conv = conv;
    jb.status = status; jb.hist = hist; jb.next = 0;
    pthread_mutex_init(&jb.lock, NULL);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > 256) nthreads = 256;
    pthread_t th[256];
    int started = 0;
    for (int t = 1; t < nthreads; t++)
        if (pthread_create(&th[started], NULL, worker, &jb) == 0) started++;
    worker(&jb);
    for (int t = 0; t < started; t++) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&jb.lock);
    return 0;
}
