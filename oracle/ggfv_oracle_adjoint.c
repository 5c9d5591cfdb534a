/*
 * ggfv_oracle_adjoint.c -- FP64 discrete adjoint of one step of eq. (3).
 *
 * TEST INFRASTRUCTURE ONLY (see ggfv_oracle.c).
 *
 * The forward step F maps x^k = (U, V, W) to x^{k+1} with the parameters
 * p = (delta1, rho2, Delta2, rho3, delta3) and the per-cell tensor (a, b, c).
 * Given lam' = dL/dx^{k+1}, this computes
 *   lam   = (dF/dx)^T lam'            (the adjoint state at level k)
 *   g_abc += (dF/d(a,b,c))^T lam'     (per-cell tensor gradients)
 *   g_p   += (dF/dp)^T lam'           (five scalar gradients)
 * with dt held fixed.  It is written in scatter form: every face flux of the
 * forward step is visited once and the chain rule of that flux is applied to
 * both cells it touches and to every value it reads (including the mirrored
 * tangential differences at the boundary).  No symmetry of the discrete
 * operators is assumed; the result is the plain transpose of the forward map.
 *
 * Face flux derivatives (x-face between l and r = l+1, s = dt*idx*(lamW_l - lamW_r)
 * is the loss sensitivity to the face flux):
 *   FX = 0.5(a_l+a_r)(W_r-W_l) idx + 0.5(b_l ty_l + b_r ty_r)
 *     dFX/dW_r = -dFX/dW_l = 0.5(a_l+a_r) idx
 *     dFX/da_l = dFX/da_r = 0.5 (W_r-W_l) idx
 *     dFX/db_l = 0.5 ty_l, dFX/db_r = 0.5 ty_r
 *     dFX/dty_l = 0.5 b_l, with ty_l = (W(l, j+1) - W(l, j-1)) hy (mirrored rows)
 *   GX = (1 - 0.5(U_l+U_r))(V_r-V_l) idx, sensitivity dt*Delta2*idx*(lamV_l - lamV_r)
 *     dGX/dV_r = -dGX/dV_l = (1 - 0.5(U_l+U_r)) idx
 *     dGX/dU_l = dGX/dU_r = -0.5 (V_r-V_l) idx
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define IX(i, j) ((size_t)(j) * (size_t)nx + (size_t)(i))

static int clampa(int k, int n)
{
    if (k < 0) return 0;
    if (k >= n) return n - 1;
    return k;
}

void orc_div_v(int nx, int ny, double lx, double ly, const double *U, const double *V, double *out);

void orc_adjoint_step(int nx, int ny, double lx, double ly, const double *prm, double dt,
                      const double *u, const double *v, const double *w, const double *a,
                      const double *b, const double *c, const double *lu1, const double *lv1,
                      const double *lw1, double *lu, double *lv, double *lw, double *ga,
                      double *gb, double *gc, double *gp)
{
    size_t n = (size_t)nx * ny;
    double d1 = prm[0], r2 = prm[1], D2 = prm[2], r3 = prm[3], d3 = prm[4];
    double idx = nx / lx, idy = ny / ly, hx = 0.5 * idx, hy = 0.5 * idy;

    /* pointwise (reaction and identity) part */
    double *dV = malloc(n * sizeof(double));
    orc_div_v(nx, ny, lx, ly, u, v, dV);
    for (size_t k = 0; k < n; ++k) {
        lu[k] = lu1[k] * (1.0 + dt * (1.0 - 2.0 * u[k] - d1 * w[k]));
        lv[k] = lv1[k] * (1.0 + dt * r2 * (1.0 - 2.0 * v[k])) + dt * r3 * lw1[k];
        lw[k] = lw1[k] * (1.0 - dt * d3) - dt * d1 * u[k] * lu1[k];
        gp[0] += -dt * u[k] * w[k] * lu1[k];
        gp[1] += dt * v[k] * (1.0 - v[k]) * lv1[k];
        gp[2] += dt * dV[k] * lv1[k];
        gp[3] += dt * v[k] * lw1[k];
        gp[4] += -dt * w[k] * lw1[k];
    }
    free(dV);

    /* x-faces */
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i + 1 < nx; ++i) {
            size_t l = IX(i, j), r = IX(i + 1, j);
            /* tumour-cell flux */
            double sv = dt * D2 * idx * (lv1[l] - lv1[r]);
            double mob = 1.0 - 0.5 * (u[l] + u[r]);
            lv[r] += sv * mob * idx;
            lv[l] -= sv * mob * idx;
            lu[l] += sv * (-0.5 * (v[r] - v[l]) * idx);
            lu[r] += sv * (-0.5 * (v[r] - v[l]) * idx);
            /* acid flux */
            double s = dt * idx * (lw1[l] - lw1[r]);
            double am = 0.5 * (a[l] + a[r]) * idx;
            lw[r] += s * am;
            lw[l] -= s * am;
            ga[l] += s * 0.5 * (w[r] - w[l]) * idx;
            ga[r] += s * 0.5 * (w[r] - w[l]) * idx;
            int jp = clampa(j + 1, ny), jm = clampa(j - 1, ny);
            double tyl = (w[IX(i, jp)] - w[IX(i, jm)]) * hy;
            double tyr = (w[IX(i + 1, jp)] - w[IX(i + 1, jm)]) * hy;
            gb[l] += s * 0.5 * tyl;
            gb[r] += s * 0.5 * tyr;
            lw[IX(i, jp)] += s * 0.5 * b[l] * hy;
            lw[IX(i, jm)] -= s * 0.5 * b[l] * hy;
            lw[IX(i + 1, jp)] += s * 0.5 * b[r] * hy;
            lw[IX(i + 1, jm)] -= s * 0.5 * b[r] * hy;
        }

    /* y-faces */
    for (int j = 0; j + 1 < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            size_t l = IX(i, j), r = IX(i, j + 1);
            double sv = dt * D2 * idy * (lv1[l] - lv1[r]);
            double mob = 1.0 - 0.5 * (u[l] + u[r]);
            lv[r] += sv * mob * idy;
            lv[l] -= sv * mob * idy;
            lu[l] += sv * (-0.5 * (v[r] - v[l]) * idy);
            lu[r] += sv * (-0.5 * (v[r] - v[l]) * idy);
            double s = dt * idy * (lw1[l] - lw1[r]);
            double cm = 0.5 * (c[l] + c[r]) * idy;
            lw[r] += s * cm;
            lw[l] -= s * cm;
            gc[l] += s * 0.5 * (w[r] - w[l]) * idy;
            gc[r] += s * 0.5 * (w[r] - w[l]) * idy;
            int ip = clampa(i + 1, nx), im = clampa(i - 1, nx);
            double txl = (w[IX(ip, j)] - w[IX(im, j)]) * hx;
            double txr = (w[IX(ip, j + 1)] - w[IX(im, j + 1)]) * hx;
            gb[l] += s * 0.5 * txl;
            gb[r] += s * 0.5 * txr;
            lw[IX(ip, j)] += s * 0.5 * b[l] * hx;
            lw[IX(im, j)] -= s * 0.5 * b[l] * hx;
            lw[IX(ip, j + 1)] += s * 0.5 * b[r] * hx;
            lw[IX(im, j + 1)] -= s * 0.5 * b[r] * hx;
        }
}

/* Chain rule of A = R(theta) diag(l1, l2) R(theta)^T:
 *   g_l1 = ga cos^2 + gc sin^2 + gb sin cos
 *   g_l2 = ga sin^2 + gc cos^2 - gb sin cos
 *   g_th = (l1 - l2) (-ga sin 2theta + gc sin 2theta + gb cos 2theta)          */
void orc_eig_backward(long n, const double *lam1, const double *lam2, const double *theta,
                      const double *ga, const double *gb, const double *gc, double *gl1,
                      double *gl2, double *gth)
{
    for (long k = 0; k < n; ++k) {
        double cs = cos(theta[k]), sn = sin(theta[k]);
        double s2 = 2.0 * sn * cs, c2 = cs * cs - sn * sn;
        gl1[k] = ga[k] * (cs * cs) + gc[k] * (sn * sn) + gb[k] * (sn * cs);
        gl2[k] = ga[k] * (sn * sn) + gc[k] * (cs * cs) - gb[k] * (sn * cs);
        gth[k] = (lam1[k] - lam2[k]) * (-ga[k] * s2 + gc[k] * s2 + gb[k] * c2);
    }
}

/* Full reverse sweep of nsteps steps from x^0, storing every state (plain, no
 * checkpointing: memory nsteps+1 states).  lam holds dL/dx^N on entry and
 * dL/dx^0 on exit; ga, gb, gc, gp are accumulated. */
void orc_step(int nx, int ny, double lx, double ly, const double *prm, double dt,
              const double *u, const double *v, const double *w, const double *a,
              const double *b, const double *c, double *un, double *vn, double *wn,
              const double *su, const double *sv, const double *sw);

void orc_adjoint_run(int nx, int ny, double lx, double ly, const double *prm, double dt,
                     long nsteps, const double *u0, const double *v0, const double *w0,
                     const double *a, const double *b, const double *c, double *lamu,
                     double *lamv, double *lamw, double *ga, double *gb, double *gc, double *gp)
{
    size_t n = (size_t)nx * ny;
    double *X = malloc((size_t)(nsteps + 1) * 3 * n * sizeof(double));
    memcpy(X, u0, n * sizeof(double));
    memcpy(X + n, v0, n * sizeof(double));
    memcpy(X + 2 * n, w0, n * sizeof(double));
    for (long s = 0; s < nsteps; ++s) {
        double *cur = X + (size_t)s * 3 * n, *nxt = X + (size_t)(s + 1) * 3 * n;
        orc_step(nx, ny, lx, ly, prm, dt, cur, cur + n, cur + 2 * n, a, b, c, nxt, nxt + n,
                 nxt + 2 * n, NULL, NULL, NULL);
    }
    double *t = malloc(3 * n * sizeof(double));
    for (long s = nsteps - 1; s >= 0; --s) {
        double *x = X + (size_t)s * 3 * n;
        orc_adjoint_step(nx, ny, lx, ly, prm, dt, x, x + n, x + 2 * n, a, b, c, lamu, lamv, lamw,
                         t, t + n, t + 2 * n, ga, gb, gc, gp);
        memcpy(lamu, t, n * sizeof(double));
        memcpy(lamv, t + n, n * sizeof(double));
        memcpy(lamw, t + 2 * n, n * sizeof(double));
    }
    free(t);
    free(X);
}

/* The same reverse sweep with the states stored only every `every` steps
 * (checkpoints x^0, x^every, x^2every, ...): each segment is recomputed from
 * its checkpoint before its adjoint steps run.  The forward step is
 * deterministic, so the recomputed states, and hence every result, are those
 * of orc_adjoint_run; memory is about nsteps/every + every states. */
void orc_run(int nx, int ny, double lx, double ly, const double *prm, double dt,
             long nsteps, double *u, double *v, double *w, const double *a,
             const double *b, const double *c, long mass_every, double *mass_log);

void orc_adjoint_run_ckpt(int nx, int ny, double lx, double ly, const double *prm, double dt,
                          long nsteps, long every, const double *u0, const double *v0,
                          const double *w0, const double *a, const double *b, const double *c,
                          double *lamu, double *lamv, double *lamw, double *ga, double *gb,
                          double *gc, double *gp)
{
    size_t n = (size_t)nx * ny;
    long nck = (nsteps + every - 1) / every;
    double *C = malloc((size_t)nck * 3 * n * sizeof(double));
    double *S = malloc((size_t)every * 3 * n * sizeof(double));
    double *t = malloc(3 * n * sizeof(double));
    if (!C || !S || !t) {
        free(C);
        free(S);
        free(t);
        return;
    }
    /* forward: checkpoint k holds x^(k*every) */
    memcpy(C, u0, n * sizeof(double));
    memcpy(C + n, v0, n * sizeof(double));
    memcpy(C + 2 * n, w0, n * sizeof(double));
    for (long k = 1; k < nck; ++k) {
        double *x = C + (size_t)k * 3 * n;
        memcpy(x, x - 3 * n, 3 * n * sizeof(double));
        orc_run(nx, ny, lx, ly, prm, dt, every, x, x + n, x + 2 * n, a, b, c, 0, NULL);
    }
    for (long k = nck - 1; k >= 0; --k) {
        long s0 = k * every, len = nsteps - s0 < every ? nsteps - s0 : every;
        /* S holds x^(s0), ..., x^(s0+len-1) */
        memcpy(S, C + (size_t)k * 3 * n, 3 * n * sizeof(double));
        for (long q = 1; q < len; ++q) {
            double *x = S + (size_t)(q - 1) * 3 * n, *y = S + (size_t)q * 3 * n;
            orc_step(nx, ny, lx, ly, prm, dt, x, x + n, x + 2 * n, a, b, c, y, y + n, y + 2 * n,
                     NULL, NULL, NULL);
        }
        for (long q = len - 1; q >= 0; --q) {
            double *x = S + (size_t)q * 3 * n;
            orc_adjoint_step(nx, ny, lx, ly, prm, dt, x, x + n, x + 2 * n, a, b, c, lamu, lamv,
                             lamw, t, t + n, t + 2 * n, ga, gb, gc, gp);
            memcpy(lamu, t, n * sizeof(double));
            memcpy(lamv, t + n, n * sizeof(double));
            memcpy(lamw, t + 2 * n, n * sizeof(double));
        }
    }
    free(t);
    free(S);
    free(C);
}
