/*
 * FP64 reference transport sweep -- test infrastructure only.
 *
 * This file belongs to the CPU oracle.  Only the tests, the smoke check and the
 * benchmark's CPU-baseline leg may load it; the HIP library never does.
 *
 * It inverts, for each discrete direction Omega_d = (mu_d, eta_d), the
 * lowest-order (piecewise-constant, degree-0) member of the upwind DG transport
 * discretisation of the spatial-discretisation section of the paper:
 *
 *     (|mu|/hx) (psi_e - psi_upwind_x) + (|eta|/hy) (psi_e - psi_upwind_y)
 *         + sigma_t,e psi_e = rhs_e
 *
 * i.e. the face matrix F_d reduces to the upwind flux and the volume matrices
 * G_j vanish for constants.  The cell loop visits cells in upwind order (i
 * ascending when mu > 0, descending otherwise; the same for j and eta), which
 * makes the lower-triangular solve a plain forward substitution -- the
 * "sweep" the source iteration of Algorithm 1, step 4 inverts each iteration.
 *
 * Inflow values on the two inflow faces are supplied by the caller per
 * direction (vacuum -> 0, isotropic inflow -> B(T_b), reflecting -> the
 * caller's lagged reflected value), so this routine holds no boundary logic.
 */
#include <math.h>

/*
 * nx, ny      cells along x and y; cell e = j*nx + i
 * hx, hy      cell widths
 * nd          number of directions
 * mu, eta     [nd] direction cosines along x and y (never exactly 0)
 * sigt        [ny*nx] total cross section sigma + 1/(c dt)
 * rhs         [nd][ny*nx] right-hand side per direction
 * inx         [nd][ny] inflow value on the x-inflow face of row j
 * iny         [nd][nx] inflow value on the y-inflow face of column i
 * psi         [nd][ny*nx] output
 */
void oracle_sweep(int nx, int ny, double hx, double hy, int nd,
                  const double *mu, const double *eta, const double *sigt,
                  const double *rhs, const double *inx, const double *iny,
                  double *psi)
{
    const long ncell = (long)nx * ny;
    for (int d = 0; d < nd; ++d) {
        const double ax = fabs(mu[d]) / hx;
        const double ay = fabs(eta[d]) / hy;
        const int sx = mu[d] > 0.0 ? 1 : -1;
        const int sy = eta[d] > 0.0 ? 1 : -1;
        const double *r = rhs + d * ncell;
        double *p = psi + d * ncell;
        for (int jj = 0; jj < ny; ++jj) {
            const int j = sy > 0 ? jj : ny - 1 - jj;
            for (int ii = 0; ii < nx; ++ii) {
                const int i = sx > 0 ? ii : nx - 1 - ii;
                const long e = (long)j * nx + i;
                const double upx = (ii == 0) ? inx[(long)d * ny + j] : p[e - sx];
                const double upy = (jj == 0) ? iny[(long)d * nx + i] : p[e - (long)sy * nx];
                p[e] = (r[e] + ax * upx + ay * upy) / (sigt[e] + ax + ay);
            }
        }
    }
}
