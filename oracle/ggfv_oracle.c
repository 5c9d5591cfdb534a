/*
 * ggfv_oracle.c -- plain FP64 CPU oracle for the explicit finite-volume step of
 * the anisotropic, heterogeneous Gatenby-Gawlinski model.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no source with the HIP path.
 *
 * What it computes (citations are to the paper's sections, equations and tables):
 *
 *   Model, Section 1, eq. (1):
 *     dU/dt = U(1-U) - d U W
 *     dV/dt = r V(1-V) + alpha div[(1-U) grad V]
 *     dW/dt = c(V-W) + div(A grad W),   A = [[a,b],[b,c]] SPD   (eq. (2))
 *   written here with delta1 = d, rho2 = r, Delta2 = alpha and the acid term
 *   generalised to rho3 V - delta3 W.
 *
 *   Scheme, Section 2, eq. (3): forward Euler, every right-hand side at level k,
 *   cell-centred unknowns on dual cells C_ij of size dx*dy, piecewise-constant
 *   tensor entries a_ij, b_ij, c_ij per cell.  The two diffusion operators are the
 *   five-point stencil of Table 1 (tumour cells) and the nine-point stencil of
 *   Table 2 (acid).  They are evaluated here in flux form: each interior face
 *   carries one flux value, the divergence is the difference of face fluxes.
 *   Expanding the flux form on an interior cell reproduces every coefficient of
 *   Tables 1 and 2 (the test suite checks this against a transcription of the
 *   tables).  Face coefficients are arithmetic means of the two cells (Section 2).
 *
 *   Neumann boundaries (Section 2, below eq. (3)): read as zero total flux through
 *   every boundary face, (A grad W).n = 0 and (1-U) grad V . n = 0.  The tangential
 *   central differences that the cross terms need in the first and last row or
 *   column take the missing neighbour as a copy of the boundary cell (the ghost
 *   copy rule U_0j = U_1j), corners mirrored in both directions.
 *
 * Arithmetic order (the same order is the contract for any other implementation,
 * so that FP64 results can agree bit for bit):
 *
 *   idx = nx/lx, idy = ny/ly, hx = 0.5*idx, hy = 0.5*idy
 *   ty(i,j) = (W(i,j+1) - W(i,j-1)) * hy        (mirrored indices)
 *   tx(i,j) = (W(i+1,j) - W(i-1,j)) * hx
 *   FX(i+1/2,j) = 0.5*(a_l + a_r) * ((W_r - W_l)*idx) + 0.5*(b_l*ty_l + b_r*ty_r)
 *   FY(i,j+1/2) = 0.5*(c_l + c_r) * ((W_r - W_l)*idy) + 0.5*(b_l*tx_l + b_r*tx_r)
 *   GX(i+1/2,j) = (1 - 0.5*(U_l + U_r)) * ((V_r - V_l)*idx), GY alike with idy
 *   divW = (FX_e - FX_w)*idx + (FY_n - FY_s)*idy,   divV alike with G
 *   U' = U + dt*( U*(1-U) - (delta1*U)*W )
 *   V' = V + dt*( (rho2*V)*(1-V) + Delta2*divV )
 *   W' = W + dt*( (rho3*V - delta3*W) + divW )
 *
 * Built with -ffp-contract=off: no fused multiply-add anywhere.
 *
 * Threads: the per-face and per-cell loops may run over rows in parallel
 * (OpenMP, when built with it).  Every value is still computed by one thread
 * from the same operands in the same order, so the results do not depend on
 * the number of threads; sums (masses, diagnostics) stay serial.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define IX(i, j) ((size_t)(j) * (size_t)nx + (size_t)(i))

static int clampi(int k, int n)
{
    if (k < 0) return 0;
    if (k >= n) return n - 1;
    return k;
}

/* Number of threads the parallel loops may use (n < 1: leave it); returns the
 * number in effect (1 without OpenMP). */
int orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
    return omp_get_max_threads();
#else
    (void)n;
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Tensor from its eigen-description: A = R(theta) diag(l1, l2) R(theta)^T,  */
/* i.e. eigenvalue l1 along (cos theta, sin theta), l2 across it (eq. (2)).   */

void orc_tensor_from_eig(long n, const double *lam1, const double *lam2,
                         const double *theta, double *a, double *b, double *c)
{
    for (long k = 0; k < n; ++k) {
        double cs = cos(theta[k]);
        double sn = sin(theta[k]);
        a[k] = lam1[k] * (cs * cs) + lam2[k] * (sn * sn);
        c[k] = lam1[k] * (sn * sn) + lam2[k] * (cs * cs);
        b[k] = (lam1[k] - lam2[k]) * (sn * cs);
    }
}

/* Largest eigenvalue of [[a,b],[b,c]]. */
double orc_lambda_max(double a, double b, double c)
{
    double m = 0.5 * (a + c);
    double d = 0.5 * (a - c);
    return m + sqrt(d * d + b * b);
}

/* Number of cells whose tensor is not positive definite (Sylvester: a > 0 and
 * a*c - b*b > 0) or not finite. */
long orc_count_not_spd(long n, const double *a, const double *b, const double *c)
{
    long bad = 0;
    for (long k = 0; k < n; ++k) {
        double det = a[k] * c[k] - b[k] * b[k];
        if (!(a[k] > 0.0) || !(det > 0.0) || !isfinite(a[k]) || !isfinite(b[k]) ||
            !isfinite(c[k]))
            ++bad;
    }
    return bad;
}

/* Explicit time-step bound used by the harness:
 *   dt = safety / (2 * max(max_ij lambda_max(A_ij), Delta2) * (idx^2 + idy^2)).
 * The step is explicit, so it is limited by the CFL condition (Section 2). */
double orc_stable_dt(int nx, int ny, double lx, double ly, const double *a,
                     const double *b, const double *c, double Delta2, double safety)
{
    double idx = nx / lx, idy = ny / ly;
    double lm = Delta2;
    for (long k = 0; k < (long)nx * ny; ++k) {
        double l = orc_lambda_max(a[k], b[k], c[k]);
        if (l > lm) lm = l;
    }
    return safety / (2.0 * lm * (idx * idx + idy * idy));
}

/* ------------------------------------------------------------------------ */
/* Diffusion operators.                                                      */

/* tangential differences with the mirrored ghost value */
static double ty_at(int nx, int ny, const double *W, int i, int j, double hy)
{
    return (W[IX(i, clampi(j + 1, ny))] - W[IX(i, clampi(j - 1, ny))]) * hy;
}

static double tx_at(int nx, int ny, const double *W, int i, int j, double hx)
{
    (void)ny;
    return (W[IX(clampi(i + 1, nx), j)] - W[IX(clampi(i - 1, nx), j)]) * hx;
}

/* D2(W; A) of eq. (3), Table 2.  out[j*nx+i] = divergence of A grad W.
 * FX[j*(nx+1) + f]: face f between cells f-1 and f; f = 0 and f = nx are the
 * domain boundary and carry zero flux.  FY[g*nx + i] likewise in y.  FX and FY
 * are work arrays of (nx+1)*ny and nx*(ny+1) values. */
static void div_w_work(int nx, int ny, double lx, double ly, const double *W, const double *a,
                       const double *b, const double *c, double *out, double *FX, double *FY)
{
    double idx = nx / lx, idy = ny / ly, hx = 0.5 * idx, hy = 0.5 * idy;
    for (int j = 0; j < ny; ++j) {
        FX[(size_t)j * (nx + 1)] = 0.0;
        FX[(size_t)j * (nx + 1) + nx] = 0.0;
    }
    for (int i = 0; i < nx; ++i) {
        FY[i] = 0.0;
        FY[(size_t)ny * nx + i] = 0.0;
    }
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i + 1 < nx; ++i) {
            size_t l = IX(i, j), r = IX(i + 1, j);
            double tyl = ty_at(nx, ny, W, i, j, hy);
            double tyr = ty_at(nx, ny, W, i + 1, j, hy);
            FX[(size_t)j * (nx + 1) + i + 1] =
                0.5 * (a[l] + a[r]) * ((W[r] - W[l]) * idx) + 0.5 * (b[l] * tyl + b[r] * tyr);
        }
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny - 1; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t l = IX(i, j), r = IX(i, j + 1);
            double txl = tx_at(nx, ny, W, i, j, hx);
            double txr = tx_at(nx, ny, W, i, j + 1, hx);
            FY[(size_t)(j + 1) * nx + i] =
                0.5 * (c[l] + c[r]) * ((W[r] - W[l]) * idy) + 0.5 * (b[l] * txl + b[r] * txr);
        }
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double fe = FX[(size_t)j * (nx + 1) + i + 1], fw = FX[(size_t)j * (nx + 1) + i];
            double fn = FY[(size_t)(j + 1) * nx + i], fs = FY[(size_t)j * nx + i];
            out[IX(i, j)] = (fe - fw) * idx + (fn - fs) * idy;
        }
}

void orc_div_w(int nx, int ny, double lx, double ly, const double *W,
               const double *a, const double *b, const double *c, double *out)
{
    double *FX = malloc((size_t)(nx + 1) * ny * sizeof(double));
    double *FY = malloc((size_t)nx * (ny + 1) * sizeof(double));
    div_w_work(nx, ny, lx, ly, W, a, b, c, out, FX, FY);
    free(FX);
    free(FY);
}

/* D1(V; U) of eq. (3), Table 1: divergence of (1-U) grad V with face mobility
 * 1 - (U_l + U_r)/2.  GX, GY: work arrays laid out as FX, FY of div_w_work. */
static void div_v_work(int nx, int ny, double lx, double ly, const double *U, const double *V,
                       double *out, double *GX, double *GY)
{
    double idx = nx / lx, idy = ny / ly;
    for (int j = 0; j < ny; ++j) {
        GX[(size_t)j * (nx + 1)] = 0.0;
        GX[(size_t)j * (nx + 1) + nx] = 0.0;
    }
    for (int i = 0; i < nx; ++i) {
        GY[i] = 0.0;
        GY[(size_t)ny * nx + i] = 0.0;
    }
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i + 1 < nx; ++i) {
            size_t l = IX(i, j), r = IX(i + 1, j);
            GX[(size_t)j * (nx + 1) + i + 1] = (1.0 - 0.5 * (U[l] + U[r])) * ((V[r] - V[l]) * idx);
        }
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny - 1; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t l = IX(i, j), r = IX(i, j + 1);
            GY[(size_t)(j + 1) * nx + i] = (1.0 - 0.5 * (U[l] + U[r])) * ((V[r] - V[l]) * idy);
        }
#pragma omp parallel for schedule(static)
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double ge = GX[(size_t)j * (nx + 1) + i + 1], gw = GX[(size_t)j * (nx + 1) + i];
            double gn = GY[(size_t)(j + 1) * nx + i], gs = GY[(size_t)j * nx + i];
            out[IX(i, j)] = (ge - gw) * idx + (gn - gs) * idy;
        }
}

void orc_div_v(int nx, int ny, double lx, double ly, const double *U, const double *V,
               double *out)
{
    double *GX = malloc((size_t)(nx + 1) * ny * sizeof(double));
    double *GY = malloc((size_t)nx * (ny + 1) * sizeof(double));
    div_v_work(nx, ny, lx, ly, U, V, out, GX, GY);
    free(GX);
    free(GY);
}

/* ------------------------------------------------------------------------ */
/* One forward-Euler step of eq. (3), from level k (u,v,w) to level k+1       */
/* (un,vn,wn).  prm = {delta1, rho2, Delta2, rho3, delta3}.  The optional     */
/* source arrays su, sv, sw (NULL for none) add dt*S after the scheme's own   */
/* update; they exist only for manufactured-solution tests.                   */

/* Work arrays of one step: divergences dW, dV (n values each) and the face
 * fluxes of both operators. */
typedef struct {
    double *dW, *dV, *FX, *FY, *GX, *GY;
} step_work;

static int work_alloc(step_work *ws, int nx, int ny)
{
    size_t n = (size_t)nx * ny, fx = (size_t)(nx + 1) * ny, fy = (size_t)nx * (ny + 1);
    ws->dW = malloc(n * sizeof(double));
    ws->dV = malloc(n * sizeof(double));
    ws->FX = malloc(fx * sizeof(double));
    ws->FY = malloc(fy * sizeof(double));
    ws->GX = malloc(fx * sizeof(double));
    ws->GY = malloc(fy * sizeof(double));
    return ws->dW && ws->dV && ws->FX && ws->FY && ws->GX && ws->GY;
}

static void work_free(step_work *ws)
{
    free(ws->dW);
    free(ws->dV);
    free(ws->FX);
    free(ws->FY);
    free(ws->GX);
    free(ws->GY);
}

static void step_work_run(int nx, int ny, double lx, double ly, const double *prm, double dt,
                          const double *u, const double *v, const double *w, const double *a,
                          const double *b, const double *c, double *un, double *vn, double *wn,
                          const double *su, const double *sv, const double *sw, step_work *ws)
{
    size_t n = (size_t)nx * ny;
    double d1 = prm[0], r2 = prm[1], D2 = prm[2], r3 = prm[3], d3 = prm[4];
    double *dW = ws->dW, *dV = ws->dV;
    div_w_work(nx, ny, lx, ly, w, a, b, c, dW, ws->FX, ws->FY);
    div_v_work(nx, ny, lx, ly, u, v, dV, ws->GX, ws->GY);
#pragma omp parallel for schedule(static)
    for (size_t k = 0; k < n; ++k) {
        double U = u[k], V = v[k], W = w[k];
        double Un = U + dt * (U * (1.0 - U) - (d1 * U) * W);
        double Vn = V + dt * ((r2 * V) * (1.0 - V) + D2 * dV[k]);
        double Wn = W + dt * ((r3 * V - d3 * W) + dW[k]);
        if (su) Un = Un + dt * su[k];
        if (sv) Vn = Vn + dt * sv[k];
        if (sw) Wn = Wn + dt * sw[k];
        un[k] = Un;
        vn[k] = Vn;
        wn[k] = Wn;
    }
}

void orc_step(int nx, int ny, double lx, double ly, const double *prm, double dt,
              const double *u, const double *v, const double *w, const double *a,
              const double *b, const double *c, double *un, double *vn, double *wn,
              const double *su, const double *sv, const double *sw)
{
    step_work ws = {0};
    if (work_alloc(&ws, nx, ny))
        step_work_run(nx, ny, lx, ly, prm, dt, u, v, w, a, b, c, un, vn, wn, su, sv, sw, &ws);
    work_free(&ws);
}

/* max over cells of the per-cell Gershgorin bound of the explicit update's
 * diffusion part:  max( 2(a idx^2 + c idy^2) + |b| idx idy,  2 Delta2 |1-u| (idx^2 + idy^2) ) */
static double gershgorin_max(int nx, int ny, double lx, double ly, const double *u, const double *a,
                             const double *b, const double *c, double Delta2)
{
    size_t n = (size_t)nx * ny;
    double idx = nx / lx, idy = ny / ly;
    double cmax = 0.0;
    for (size_t k = 0; k < n; ++k) {
        double cw = 2.0 * (a[k] * (idx * idx) + c[k] * (idy * idy)) + fabs(b[k]) * (idx * idy);
        double cv = 2.0 * Delta2 * fabs(1.0 - u[k]) * (idx * idx + idy * idy);
        if (cw > cmax) cmax = cw;
        if (cv > cmax) cmax = cv;
    }
    return cmax;
}

/* Diagnostics of a state (row-major serial sums):
 *   out[0..2]  mass of u, v, w = dx*dy*sum
 *   out[3..5]  min of u, v, w over finite values
 *   out[6..8]  max of u, v, w over finite values
 *   out[9]     cfl = dt * max_ij max( 2(a idx^2 + c idy^2) + |b| idx idy,
 *                                     2 Delta2 |1-u| (idx^2 + idy^2) )
 *              (the per-cell Gershgorin bound of the explicit update; the
 *              step is stable when it stays at or below 1)
 *   out[10]    number of non-finite values among u, v, w                       */
void orc_diag(int nx, int ny, double lx, double ly, const double *u, const double *v,
              const double *w, const double *a, const double *b, const double *c,
              double Delta2, double dt, double *out)
{
    size_t n = (size_t)nx * ny;
    double dx = lx / nx, dy = ly / ny;
    const double *f[3] = {u, v, w};
    double nonfinite = 0.0;
    for (int q = 0; q < 3; ++q) {
        double s = 0.0, mn = INFINITY, mx = -INFINITY;
        for (size_t k = 0; k < n; ++k) {
            double x = f[q][k];
            if (!isfinite(x)) {
                nonfinite += 1.0;
                continue;
            }
            s += x;
            if (x < mn) mn = x;
            if (x > mx) mx = x;
        }
        out[q] = dx * dy * s;
        out[3 + q] = mn;
        out[6 + q] = mx;
    }
    out[9] = dt * gershgorin_max(nx, ny, lx, ly, u, a, b, c, Delta2);
    out[10] = nonfinite;
}

/* Adaptive step size.  Section 2 chooses a new step size Delta t_k after every
 * iteration so that the explicit scheme stays stable, without printing the
 * rule.  Reading: the largest dt whose per-cell Gershgorin number (the cfl of
 * orc_diag, on the current state) equals `safety`:
 *   dt_k = safety / max_ij max( 2(a idx^2 + c idy^2) + |b| idx idy,
 *                               2 Delta2 |1-u_ij^k| (idx^2 + idy^2) ).
 * The first term is the acid diffusion (Table 2), the second the tumour-cell
 * diffusion with its mobility 1-u (Table 1) on the current normal-cell density. */
double orc_adaptive_dt(int nx, int ny, double lx, double ly, const double *u, const double *a,
                       const double *b, const double *c, double Delta2, double safety)
{
    return safety / gershgorin_max(nx, ny, lx, ly, u, a, b, c, Delta2);
}

/* nsteps adaptive steps in place on (u, v, w): before every step the step size
 * is orc_adaptive_dt of the current state; it is written to dt_log[k] (if not
 * NULL) and added to *t (t_{k+1} = t_k + dt_k). */
void orc_run_adaptive(int nx, int ny, double lx, double ly, const double *prm, double safety,
                      long nsteps, double *u, double *v, double *w, const double *a,
                      const double *b, const double *c, double *dt_log, double *t)
{
    size_t n = (size_t)nx * ny;
    double *un = malloc(n * sizeof(double));
    double *vn = malloc(n * sizeof(double));
    double *wn = malloc(n * sizeof(double));
    for (long s = 0; s < nsteps; ++s) {
        double dt = orc_adaptive_dt(nx, ny, lx, ly, u, a, b, c, prm[2], safety);
        orc_step(nx, ny, lx, ly, prm, dt, u, v, w, a, b, c, un, vn, wn, NULL, NULL, NULL);
        memcpy(u, un, n * sizeof(double));
        memcpy(v, vn, n * sizeof(double));
        memcpy(w, wn, n * sizeof(double));
        if (dt_log) dt_log[s] = dt;
        *t += dt;
    }
    free(un);
    free(vn);
    free(wn);
}

/* Front diagnostics for fronts that advance towards +x (Section 2's
 * propagating tumour fronts and the interstitial gap between the tumour and the
 * healthy tissue).  The paper prints no definition; reading, per row j:
 *   tumour front  xv_j: the largest cell index i with v_ij >= theta_v, moved to
 *                 the threshold crossing by linear interpolation towards cell
 *                 i+1 (x_i + (v_i - theta_v)/(v_i - v_i+1) dx when cell i+1
 *                 exists and lies below the threshold; x_i otherwise);
 *   tissue front  xu_j: the smallest index i beyond the tumour front's cell
 *                 with u_ij >= theta_u, moved back to the crossing by linear
 *                 interpolation towards cell i-1 (x_i - (u_i - theta_u)/(u_i -
 *                 u_i-1) dx when u_i-1 < theta_u);
 *   gap           g_j = xu_j - xv_j (the width of the region between the two
 *                 fronts where neither population reaches its threshold).
 * Cell centres are x_i = (i + 1/2) dx.  A row has a tumour front if some cell
 * reaches theta_v, and a gap if it also has a tissue front.  Outputs:
 *   out[0..2]  mean, min, max of xv over rows with a tumour front
 *   out[3..5]  mean, min, max of xu over rows with a gap
 *   out[6..8]  mean, min, max of g over rows with a gap
 *   out[9], out[10]  number of rows with a tumour front, with a gap
 * (means are serial sums in row order divided by the count; 0 when the count
 * is 0, min and max then +inf and -inf). */
void orc_front_diag(int nx, int ny, double lx, const double *u, const double *v, double theta_u,
                    double theta_v, double *out)
{
    double dx = lx / nx;
    double s[3] = {0.0, 0.0, 0.0}, mn[3], mx[3];
    long nv = 0, ng = 0;
    for (int q = 0; q < 3; ++q) {
        mn[q] = INFINITY;
        mx[q] = -INFINITY;
    }
    for (int j = 0; j < ny; ++j) {
        int iv = -1;
        for (int i = 0; i < nx; ++i)
            if (v[IX(i, j)] >= theta_v) iv = i;
        if (iv < 0) continue;
        double xv = (iv + 0.5) * dx;
        if (iv + 1 < nx) {
            double a = v[IX(iv, j)], b = v[IX(iv + 1, j)];
            xv = xv + (a - theta_v) / (a - b) * dx;
        }
        ++nv;
        s[0] += xv;
        if (xv < mn[0]) mn[0] = xv;
        if (xv > mx[0]) mx[0] = xv;
        int iu = -1;
        for (int i = iv + 1; i < nx; ++i)
            if (u[IX(i, j)] >= theta_u) {
                iu = i;
                break;
            }
        if (iu < 0) continue;
        double xu = (iu + 0.5) * dx;
        double c = u[IX(iu, j)], d = u[IX(iu - 1, j)];
        if (d < theta_u) xu = xu - (c - theta_u) / (c - d) * dx;
        double g = xu - xv;
        ++ng;
        s[1] += xu;
        s[2] += g;
        if (xu < mn[1]) mn[1] = xu;
        if (xu > mx[1]) mx[1] = xu;
        if (g < mn[2]) mn[2] = g;
        if (g > mx[2]) mx[2] = g;
    }
    out[0] = nv > 0 ? s[0] / (double)nv : 0.0;
    out[3] = ng > 0 ? s[1] / (double)ng : 0.0;
    out[6] = ng > 0 ? s[2] / (double)ng : 0.0;
    for (int q = 0; q < 3; ++q) {
        out[3 * q + 1] = mn[q];
        out[3 * q + 2] = mx[q];
    }
    out[9] = (double)nv;
    out[10] = (double)ng;
}

/* Speed of a front from two masses (LeVeque and Yee's space-averaged wave
 * speed, cited in Section 2): a front that moves the transition between the
 * state behind it (density `behind`) and the state ahead of it (`ahead`) by
 * s*(t1 - t0) across a domain of height ly changes the mass by
 * ly*(behind - ahead)*s*(t1 - t0). */
double orc_front_speed(double mass0, double mass1, double t0, double t1, double ly, double behind,
                       double ahead)
{
    return (mass1 - mass0) / ((t1 - t0) * ly * (behind - ahead));
}

/* nsteps steps in place on (u, v, w).  When mass_every > 0, the masses of u, v, w
 * after every mass_every-th step are written to mass_log (3 per entry). */
void orc_run(int nx, int ny, double lx, double ly, const double *prm, double dt,
             long nsteps, double *u, double *v, double *w, const double *a,
             const double *b, const double *c, long mass_every, double *mass_log)
{
    size_t n = (size_t)nx * ny;
    /* two levels: the caller's arrays and one more; the levels alternate and
     * the last one is copied back into the caller's arrays */
    double *lev[2][3] = {{u, v, w}, {malloc(n * sizeof(double)), malloc(n * sizeof(double)),
                                     malloc(n * sizeof(double))}};
    step_work ws = {0};
    double dg[11];
    long logged = 0;
    int cur = 0;
    int ok = lev[1][0] && lev[1][1] && lev[1][2] && work_alloc(&ws, nx, ny);
    for (long s = 0; ok && s < nsteps; ++s) {
        double **x = lev[cur], **y = lev[1 - cur];
        step_work_run(nx, ny, lx, ly, prm, dt, x[0], x[1], x[2], a, b, c, y[0], y[1], y[2], NULL, NULL, NULL,
                      &ws);
        cur = 1 - cur;
        if (mass_every > 0 && mass_log && (s + 1) % mass_every == 0) {
            orc_diag(nx, ny, lx, ly, y[0], y[1], y[2], a, b, c, prm[2], dt, dg);
            mass_log[3 * logged + 0] = dg[0];
            mass_log[3 * logged + 1] = dg[1];
            mass_log[3 * logged + 2] = dg[2];
            ++logged;
        }
    }
    work_free(&ws);
    if (cur == 1)
        for (int q = 0; q < 3; ++q) memcpy(lev[0][q], lev[1][q], n * sizeof(double));
    for (int q = 0; q < 3; ++q) free(lev[1][q]);
}
