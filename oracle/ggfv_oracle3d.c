/*
 * ggfv_oracle3d.c -- plain FP64 CPU oracle for the three-dimensional form of the
 * explicit finite-volume step.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the test suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no source with the HIP path.
 *
 * The model of Section 1 (eq. (1)) is stated for a domain of dimension 2 or 3,
 * and the paper's outlook is three-dimensional modelling; it prints no 3D
 * scheme.  Reading: the scheme of Section 2 (eq. (3)) with the same flux form in
 * three directions, on cells of size dx*dy*dz:
 *
 *   tensor per cell  A = [[axx, axy, axz], [axy, ayy, ayz], [axz, ayz, azz]]
 *   tx = (W(i+1) - W(i-1)) * hx,  ty, tz alike   (mirrored indices, h = idx/2)
 *   FX(i+1/2) = 0.5*(axx_l + axx_r) * ((W_r - W_l)*idx)
 *             + 0.5*(axy_l*ty_l + axy_r*ty_r) + 0.5*(axz_l*tz_l + axz_r*tz_r)
 *   FY(j+1/2) = 0.5*(ayy_l + ayy_r) * ((W_r - W_l)*idy)
 *             + 0.5*(axy_l*tx_l + axy_r*tx_r) + 0.5*(ayz_l*tz_l + ayz_r*tz_r)
 *   FZ(k+1/2) = 0.5*(azz_l + azz_r) * ((W_r - W_l)*idz)
 *             + 0.5*(axz_l*tx_l + axz_r*tx_r) + 0.5*(ayz_l*ty_l + ayz_r*ty_r)
 *   GX = (1 - 0.5*(U_l + U_r)) * ((V_r - V_l)*idx),  GY, GZ alike
 *   divW = ((FX_e - FX_w)*idx + (FY_n - FY_s)*idy) + (FZ_t - FZ_b)*idz,  divV alike
 *   U' = U + dt*( U*(1-U) - (delta1*U)*W )
 *   V' = V + dt*( (rho2*V)*(1-V) + Delta2*divV )
 *   W' = W + dt*( (rho3*V - delta3*W) + divW )
 * (sums evaluated left to right as written).  The acid flux couples each cell
 * to 18 neighbours (the 19-point stencil: faces and edges, no corners), the
 * tumour-cell flux to its 6 face neighbours.  Boundary faces carry zero flux;
 * tangential differences take the boundary cell as its missing neighbour.
 * With nz = 1 and axz = ayz = 0 every z term vanishes and the 2D scheme results.
 *
 * Built with -ffp-contract=off: no fused multiply-add anywhere.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define IX3(i, j, k) (((size_t)(k) * (size_t)ny + (size_t)(j)) * (size_t)nx + (size_t)(i))

static int clamp3(int k, int n)
{
    if (k < 0) return 0;
    if (k >= n) return n - 1;
    return k;
}

/* tangential central differences with the mirrored ghost value */
static double t3x(int nx, int ny, const double *W, int i, int j, int k, double hx)
{
    return (W[IX3(clamp3(i + 1, nx), j, k)] - W[IX3(clamp3(i - 1, nx), j, k)]) * hx;
}

static double t3y(int nx, int ny, const double *W, int i, int j, int k, double hy)
{
    return (W[IX3(i, clamp3(j + 1, ny), k)] - W[IX3(i, clamp3(j - 1, ny), k)]) * hy;
}

static double t3z(int nx, int ny, int nz, const double *W, int i, int j, int k, double hz)
{
    return (W[IX3(i, j, clamp3(k + 1, nz))] - W[IX3(i, j, clamp3(k - 1, nz))]) * hz;
}

/* div(A grad W) of the 3D scheme.  A = {axx, ayy, azz, axy, axz, ayz}, each a
 * full field.  out is indexed like W. */
void orc3_div_w(int nx, int ny, int nz, double lx, double ly, double lz, const double *W,
                const double *const *A, double *out)
{
    const double *axx = A[0], *ayy = A[1], *azz = A[2], *axy = A[3], *axz = A[4], *ayz = A[5];
    double idx = nx / lx, idy = ny / ly, idz = nz / lz;
    double hx = 0.5 * idx, hy = 0.5 * idy, hz = 0.5 * idz;
    size_t n = (size_t)nx * ny * nz;
    /* face fluxes: FX[c] is the face between cell c and its +x neighbour (zero on
     * the last column), FY and FZ alike */
    double *FX = calloc(n, sizeof(double));
    double *FY = calloc(n, sizeof(double));
    double *FZ = calloc(n, sizeof(double));
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t l = IX3(i, j, k);
                if (i + 1 < nx) {
                    size_t r = IX3(i + 1, j, k);
                    double tyl = t3y(nx, ny, W, i, j, k, hy), tyr = t3y(nx, ny, W, i + 1, j, k, hy);
                    double tzl = t3z(nx, ny, nz, W, i, j, k, hz), tzr = t3z(nx, ny, nz, W, i + 1, j, k, hz);
                    FX[l] = 0.5 * (axx[l] + axx[r]) * ((W[r] - W[l]) * idx) +
                            0.5 * (axy[l] * tyl + axy[r] * tyr) + 0.5 * (axz[l] * tzl + axz[r] * tzr);
                }
                if (j + 1 < ny) {
                    size_t r = IX3(i, j + 1, k);
                    double txl = t3x(nx, ny, W, i, j, k, hx), txr = t3x(nx, ny, W, i, j + 1, k, hx);
                    double tzl = t3z(nx, ny, nz, W, i, j, k, hz), tzr = t3z(nx, ny, nz, W, i, j + 1, k, hz);
                    FY[l] = 0.5 * (ayy[l] + ayy[r]) * ((W[r] - W[l]) * idy) +
                            0.5 * (axy[l] * txl + axy[r] * txr) + 0.5 * (ayz[l] * tzl + ayz[r] * tzr);
                }
                if (k + 1 < nz) {
                    size_t r = IX3(i, j, k + 1);
                    double txl = t3x(nx, ny, W, i, j, k, hx), txr = t3x(nx, ny, W, i, j, k + 1, hx);
                    double tyl = t3y(nx, ny, W, i, j, k, hy), tyr = t3y(nx, ny, W, i, j, k + 1, hy);
                    FZ[l] = 0.5 * (azz[l] + azz[r]) * ((W[r] - W[l]) * idz) +
                            0.5 * (axz[l] * txl + axz[r] * txr) + 0.5 * (ayz[l] * tyl + ayz[r] * tyr);
                }
            }
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = IX3(i, j, k);
                double fw = i > 0 ? FX[IX3(i - 1, j, k)] : 0.0;
                double fs = j > 0 ? FY[IX3(i, j - 1, k)] : 0.0;
                double fb = k > 0 ? FZ[IX3(i, j, k - 1)] : 0.0;
                out[c] = ((FX[c] - fw) * idx + (FY[c] - fs) * idy) + (FZ[c] - fb) * idz;
            }
    free(FX);
    free(FY);
    free(FZ);
}

/* div((1-U) grad V) of the 3D scheme (face mobility 1 - (U_l + U_r)/2). */
void orc3_div_v(int nx, int ny, int nz, double lx, double ly, double lz, const double *U,
                const double *V, double *out)
{
    double idx = nx / lx, idy = ny / ly, idz = nz / lz;
    size_t n = (size_t)nx * ny * nz;
    double *GX = calloc(n, sizeof(double));
    double *GY = calloc(n, sizeof(double));
    double *GZ = calloc(n, sizeof(double));
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t l = IX3(i, j, k);
                if (i + 1 < nx) {
                    size_t r = IX3(i + 1, j, k);
                    GX[l] = (1.0 - 0.5 * (U[l] + U[r])) * ((V[r] - V[l]) * idx);
                }
                if (j + 1 < ny) {
                    size_t r = IX3(i, j + 1, k);
                    GY[l] = (1.0 - 0.5 * (U[l] + U[r])) * ((V[r] - V[l]) * idy);
                }
                if (k + 1 < nz) {
                    size_t r = IX3(i, j, k + 1);
                    GZ[l] = (1.0 - 0.5 * (U[l] + U[r])) * ((V[r] - V[l]) * idz);
                }
            }
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                size_t c = IX3(i, j, k);
                double gw = i > 0 ? GX[IX3(i - 1, j, k)] : 0.0;
                double gs = j > 0 ? GY[IX3(i, j - 1, k)] : 0.0;
                double gb = k > 0 ? GZ[IX3(i, j, k - 1)] : 0.0;
                out[c] = ((GX[c] - gw) * idx + (GY[c] - gs) * idy) + (GZ[c] - gb) * idz;
            }
    free(GX);
    free(GY);
    free(GZ);
}

/* One forward-Euler step of the 3D scheme from (u,v,w) to (un,vn,wn);
 * prm = {delta1, rho2, Delta2, rho3, delta3}. */
void orc3_step(int nx, int ny, int nz, double lx, double ly, double lz, const double *prm, double dt,
               const double *u, const double *v, const double *w, const double *const *A, double *un,
               double *vn, double *wn)
{
    size_t n = (size_t)nx * ny * nz;
    double d1 = prm[0], r2 = prm[1], D2 = prm[2], r3 = prm[3], d3 = prm[4];
    double *dW = malloc(n * sizeof(double));
    double *dV = malloc(n * sizeof(double));
    orc3_div_w(nx, ny, nz, lx, ly, lz, w, A, dW);
    orc3_div_v(nx, ny, nz, lx, ly, lz, u, v, dV);
    for (size_t c = 0; c < n; ++c) {
        double U = u[c], V = v[c], W = w[c];
        un[c] = U + dt * (U * (1.0 - U) - (d1 * U) * W);
        vn[c] = V + dt * ((r2 * V) * (1.0 - V) + D2 * dV[c]);
        wn[c] = W + dt * ((r3 * V - d3 * W) + dW[c]);
    }
    free(dW);
    free(dV);
}

/* nsteps steps in place. */
void orc3_run(int nx, int ny, int nz, double lx, double ly, double lz, const double *prm, double dt,
              long nsteps, double *u, double *v, double *w, const double *const *A)
{
    size_t n = (size_t)nx * ny * nz;
    double *un = malloc(n * sizeof(double));
    double *vn = malloc(n * sizeof(double));
    double *wn = malloc(n * sizeof(double));
    for (long s = 0; s < nsteps; ++s) {
        orc3_step(nx, ny, nz, lx, ly, lz, prm, dt, u, v, w, A, un, vn, wn);
        memcpy(u, un, n * sizeof(double));
        memcpy(v, vn, n * sizeof(double));
        memcpy(w, wn, n * sizeof(double));
    }
    free(un);
    free(vn);
    free(wn);
}

/* Explicit step bound of the 3D scheme: the largest eigenvalue of each cell's
 * tensor is bounded by its largest absolute row sum (Gershgorin), so
 *   dt = safety / (2 * max(max_cells G, Delta2) * (idx^2 + idy^2 + idz^2)),
 *   G = max(|axx| + |axy| + |axz|, |axy| + |ayy| + |ayz|, |axz| + |ayz| + |azz|). */
double orc3_stable_dt(int nx, int ny, int nz, double lx, double ly, double lz, const double *const *A,
                      double Delta2, double safety)
{
    const double *axx = A[0], *ayy = A[1], *azz = A[2], *axy = A[3], *axz = A[4], *ayz = A[5];
    double idx = nx / lx, idy = ny / ly, idz = nz / lz;
    double g = Delta2;
    size_t n = (size_t)nx * ny * nz;
    for (size_t c = 0; c < n; ++c) {
        double r0 = fabs(axx[c]) + fabs(axy[c]) + fabs(axz[c]);
        double r1 = fabs(axy[c]) + fabs(ayy[c]) + fabs(ayz[c]);
        double r2 = fabs(axz[c]) + fabs(ayz[c]) + fabs(azz[c]);
        if (r0 > g) g = r0;
        if (r1 > g) g = r1;
        if (r2 > g) g = r2;
    }
    return safety / (2.0 * g * (idx * idx + idy * idy + idz * idz));
}

/* Masses (dx*dy*dz*sum, serial order) of u, v, w into out[0..2]. */
void orc3_mass(int nx, int ny, int nz, double lx, double ly, double lz, const double *u, const double *v,
               const double *w, double *out)
{
    size_t n = (size_t)nx * ny * nz;
    double vol = (lx / nx) * (ly / ny) * (lz / nz);
    const double *f[3] = {u, v, w};
    for (int q = 0; q < 3; ++q) {
        double s = 0.0;
        for (size_t c = 0; c < n; ++c) s += f[q][c];
        out[q] = vol * s;
    }
}
