/*
 * Plain FP64 CPU oracle for the second-order Trotter-Suzuki time step of one
 * particle on a 2D real-space mesh (Wittek & Cucchietti, "A Second-Order
 * Distributed Trotter-Suzuki Solver with a Hybrid Kernel", Sec. 2).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant with the HIP
 * library.  It is deliberately slow and literal: every sweep is a separate
 * pass over the whole mesh, steps are never merged, nothing is blocked.
 *
 * Conventions (readings of the paper, each argued in the design notes):
 *   - i hbar dpsi/dt = H psi, so one step approximates exp(-i dt H / hbar)
 *     (Sec. 2, Eq. "evolution"; the printed sign of Eq. "schrodinger" is at
 *     odds with it and the solution's sign is taken).
 *   - H = H0 + (even pairs) + (odd pairs) per axis (Sec. 2, the H0/H1/H2
 *     split, extended to two dimensions as the five-part split of Sec. 2).
 *     The tunnelling element between neighbours is -J_a with
 *     J_a = hbar^2 / (2 m da^2); the diagonal is
 *     eps_l = V_l + hbar^2/(m dx^2) + hbar^2/(m dy^2).
 *   - The exponential of one 2x2 block [[0,-J],[-J,0]] acting for time tau is
 *     [[c, i s], [i s, c]] with c = cos(alpha), s = sin(alpha),
 *     alpha = tau J / hbar (the paper prints -i s; with its own negative
 *     tunnelling element and the solution's sign the off-diagonal is +i s).
 *     The rotation is evaluated in the delta form
 *         a' = a + (i s b - d a),  b' = b + (i s a - d b),
 *     with d = 1 - c = 2 sin^2(alpha/2), the same number written without the
 *     cancellation of 1 - cos.
 *   - U2(dt) is the symmetrised product of first-order factors each acting
 *     for dt/2 (Sec. 2, Eq. "secondorder", read as the standard
 *     symmetrisation; the printed form would evolve for 2 dt).  In the order
 *     the factors are applied to the state:
 *         Ox(h) Oy(h) Ex(h) Ey(h) P(dt) Ey(h) Ex(h) Oy(h) Ox(h),  h = dt/2,
 *     where E/O rotate the even pairs (2j,2j+1) / odd pairs (2j+1,2j+2) of
 *     every line along that axis and P multiplies by exp(-i dt eps_l/hbar).
 *   - Periodic boundaries (the odd set holds the wrap pair (L-1, 0); sides
 *     must be even) or closed boundaries (no wrap pair; sides of any length
 *     >= 2; the diagonal keeps its full value at the walls).
 *
 * Layout: psi is (ny, nx) row-major, x fastest, interleaved (re, im) doubles.
 * V is (ny, nx) doubles.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define TSO_BC_PERIODIC 0
#define TSO_BC_CLOSED 1

/* ---- argument checks -------------------------------------------------- */

static int sides_ok(int nx, int ny, int bc) {
    if (nx < 2 || ny < 2) return 0;
    if (bc == TSO_BC_PERIODIC) return (nx % 2 == 0) && (ny % 2 == 0);
    if (bc == TSO_BC_CLOSED) return 1;
    return 0;
}

static int params_ok(double dx, double dy, double mass, double hbar) {
    return isfinite(dx) && isfinite(dy) && isfinite(mass) && isfinite(hbar) &&
           dx > 0 && dy > 0 && mass > 0 && hbar > 0;
}

void tso_set_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int tso_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ---- one 2x2 block: exp(-i tau [[0,-J],[-J,0]] / hbar) on (a, b) ------ */

static void rotate(double *a, double *b, double s, double d) {
    double ar = a[0], ai = a[1], br = b[0], bi = b[1];
    /* i s b = (-s bi) + i (s br) */
    a[0] = ar + (-s * bi - d * ar);
    a[1] = ai + (s * br - d * ai);
    b[0] = br + (-s * ai - d * br);
    b[1] = bi + (s * ar - d * bi);
}

/* Coefficients of the block exponential for hopping energy J acting for tau. */
static void block_coeffs(double tau, double J, double hbar, double *s, double *d) {
    double alpha = tau * J / hbar;
    double half = sin(0.5 * alpha);
    *s = sin(alpha);
    *d = 2.0 * half * half;
}

/* ---- sweeps: every pair of one parity along one axis ----------------- */

/* Pairs (j, j+1) along x with j = parity (mod 2), in every row. */
static void sweep_x(int nx, int ny, int bc, int parity, double s, double d, double *psi) {
    int y;
#pragma omp parallel for schedule(static)
    for (y = 0; y < ny; ++y) {
        double *row = psi + 2 * (size_t)y * (size_t)nx;
        for (int j = parity; j < nx; j += 2) {
            int k = j + 1;
            if (k == nx) {
                if (bc == TSO_BC_CLOSED) continue;
                k = 0;
            }
            rotate(row + 2 * (size_t)j, row + 2 * (size_t)k, s, d);
        }
    }
}

/* Pairs of rows (j, j+1) with j = parity (mod 2); every column. */
static void sweep_y(int nx, int ny, int bc, int parity, double s, double d, double *psi) {
    int npairs = (ny - parity + 1) / 2;
    int p;
#pragma omp parallel for schedule(static)
    for (p = 0; p < npairs; ++p) {
        int j = parity + 2 * p;
        int k = j + 1;
        if (k == ny) {
            if (bc == TSO_BC_CLOSED) continue;
            k = 0;
        }
        double *rj = psi + 2 * (size_t)j * (size_t)nx;
        double *rk = psi + 2 * (size_t)k * (size_t)nx;
        for (int x = 0; x < nx; ++x) rotate(rj + 2 * (size_t)x, rk + 2 * (size_t)x, s, d);
    }
}

/* ---- diagonal part: psi_l <- exp(-i dt eps_l / hbar) psi_l ------------- */

static void potential_phase(int nx, int ny, double dt, double eps0, double hbar,
                            const double *V, double *psi) {
    size_t n = (size_t)nx * (size_t)ny;
    long long l;
#pragma omp parallel for schedule(static)
    for (l = 0; l < (long long)n; ++l) {
        double phi = dt * (V[l] + eps0) / hbar;
        double c = cos(phi), s = sin(phi);
        double re = psi[2 * l], im = psi[2 * l + 1];
        /* (re + i im)(c - i s) */
        psi[2 * l] = re * c + im * s;
        psi[2 * l + 1] = im * c - re * s;
    }
}

/* One second-order step U2(dt) applied to psi, in the order of Sec. 2. */
static void u2_step(int nx, int ny, int bc, double dx, double dy, double mass, double hbar,
                    double dt, const double *V, double *psi) {
    double h = 0.5 * dt;
    double Jx = hbar * hbar / (2.0 * mass * dx * dx);
    double Jy = hbar * hbar / (2.0 * mass * dy * dy);
    double eps0 = hbar * hbar / (mass * dx * dx) + hbar * hbar / (mass * dy * dy);
    double sx, dxc, sy, dyc;
    block_coeffs(h, Jx, hbar, &sx, &dxc);
    block_coeffs(h, Jy, hbar, &sy, &dyc);

    sweep_x(nx, ny, bc, 1, sx, dxc, psi);  /* Ox(h) */
    sweep_y(nx, ny, bc, 1, sy, dyc, psi);  /* Oy(h) */
    sweep_x(nx, ny, bc, 0, sx, dxc, psi);  /* Ex(h) */
    sweep_y(nx, ny, bc, 0, sy, dyc, psi);  /* Ey(h) */
    potential_phase(nx, ny, dt, eps0, hbar, V, psi);
    sweep_y(nx, ny, bc, 0, sy, dyc, psi);  /* Ey(h) */
    sweep_x(nx, ny, bc, 0, sx, dxc, psi);  /* Ex(h) */
    sweep_y(nx, ny, bc, 1, sy, dyc, psi);  /* Oy(h) */
    sweep_x(nx, ny, bc, 1, sx, dxc, psi);  /* Ox(h) */
}

/*
 * Evolve psi in place by `steps` applications of the order-`order` operator.
 *   order 2: U2(dt) per step (Sec. 2, Eq. "secondorder").
 *   order 4: U4(dt) = U2(p dt) U2(p dt) U2((1-4p) dt) U2(p dt) U2(p dt),
 *            p = 1/(4 - 4^(1/3))  (Sec. 2, Eq. "fourthorder").
 * Returns 0 on success, -1 on a bad argument (psi untouched).
 */
int tso_evolve(int nx, int ny, int bc, double dx, double dy, double mass, double hbar,
               double dt, const double *V, double *psi, long long steps, int order) {
    if (!sides_ok(nx, ny, bc) || !params_ok(dx, dy, mass, hbar) || !isfinite(dt) ||
        steps < 0 || V == NULL || psi == NULL || (order != 2 && order != 4))
        return -1;
    if (order == 2) {
        for (long long n = 0; n < steps; ++n)
            u2_step(nx, ny, bc, dx, dy, mass, hbar, dt, V, psi);
    } else {
        double p = 1.0 / (4.0 - cbrt(4.0));
        double sub[5] = {p * dt, p * dt, (1.0 - 4.0 * p) * dt, p * dt, p * dt};
        for (long long n = 0; n < steps; ++n)
            for (int k = 0; k < 5; ++k)
                u2_step(nx, ny, bc, dx, dy, mass, hbar, sub[k], V, psi);
    }
    return 0;
}

/*
 * Time-dependent potential V(t) = V0 + f(t) W.  The paper builds the product
 * for a time-independent H and notes that the time-dependent form is the same
 * construction (Sec. 2, footnote to Eq. "evolution", citing Poulin et al.):
 * step n, from t_n to t_n + dt, is U2(dt) with H frozen at the step's
 * midpoint, which keeps the product second order for smooth f.  The caller
 * gives f[n] = f(t_n + dt/2) for n = 0 .. steps-1; the potential of step n is
 * V0 + f[n] W.  Order 2 only.  Returns 0, or -1 on a bad argument (psi
 * untouched).
 */
int tso_evolve_td(int nx, int ny, int bc, double dx, double dy, double mass, double hbar,
                  double dt, const double *V0, const double *W, const double *f, double *psi,
                  long long steps) {
    if (!sides_ok(nx, ny, bc) || !params_ok(dx, dy, mass, hbar) || !isfinite(dt) ||
        steps < 0 || V0 == NULL || W == NULL || psi == NULL || (steps > 0 && f == NULL))
        return -1;
    for (long long n = 0; n < steps; ++n)
        if (!isfinite(f[n])) return -1;
    size_t sites = (size_t)nx * (size_t)ny;
    double *Vn = (double *)malloc(sites * sizeof(double));
    if (!Vn) return -1;
    for (long long n = 0; n < steps; ++n) {
        long long l;
#pragma omp parallel for schedule(static)
        for (l = 0; l < (long long)sites; ++l) Vn[l] = V0[l] + f[n] * W[l];
        u2_step(nx, ny, bc, dx, dy, mass, hbar, dt, Vn, psi);
    }
    free(Vn);
    return 0;
}

/* ---- three dimensions ------------------------------------------------- */
/*
 * The extension to three-dimensional meshes that the paper names as future
 * work (Sec. 5): the same split with a third axis, i.e. seven parts, the
 * diagonal and the even and odd pairs along x, y and z.  One step, in the
 * order the factors are applied:
 *     Ox(h) Oy(h) Oz(h) Ex(h) Ey(h) Ez(h) P(dt) Ez(h) Ey(h) Ex(h) Oz(h) Oy(h) Ox(h)
 * with eps_l = V_l + hbar^2/(m dx^2) + hbar^2/(m dy^2) + hbar^2/(m dz^2).
 * Layout (nz, ny, nx), x fastest.
 */

static void sweep3(int nx, int ny, int nz, int bc, int axis, int parity, double s, double d,
                   double *psi) {
    int L = axis == 0 ? nx : (axis == 1 ? ny : nz);
    size_t stride = axis == 0 ? 1 : (axis == 1 ? (size_t)nx : (size_t)nx * (size_t)ny);
    /* every line along `axis`: the other two coordinates */
    long long lines = (long long)nx * ny * nz / L;
    long long q;
#pragma omp parallel for schedule(static)
    for (q = 0; q < lines; ++q) {
        size_t base;
        if (axis == 0) {
            base = (size_t)q * (size_t)nx;                       /* (z, y) rows */
        } else if (axis == 1) {
            long long z = q / nx, x = q % nx;                    /* (z, x) columns */
            base = (size_t)z * (size_t)nx * (size_t)ny + (size_t)x;
        } else {
            base = (size_t)q;                                    /* (y, x) columns */
        }
        for (int j = parity; j < L; j += 2) {
            int k = j + 1;
            if (k == L) {
                if (bc == TSO_BC_CLOSED) continue;
                k = 0;
            }
            rotate(psi + 2 * (base + (size_t)j * stride), psi + 2 * (base + (size_t)k * stride), s, d);
        }
    }
}

/* Evolve psi (nz, ny, nx) in place by `steps` second-order steps; sides >= 2,
 * even under periodic boundaries.  Returns 0, or -1 on a bad argument. */
int tso_evolve3(int nx, int ny, int nz, int bc, double dx, double dy, double dz, double mass,
                double hbar, double dt, const double *V, double *psi, long long steps) {
    if (!sides_ok(nx, ny, bc) || !sides_ok(nz, 2, bc) || !params_ok(dx, dy, mass, hbar) ||
        !(isfinite(dz) && dz > 0) || !isfinite(dt) || steps < 0 || V == NULL || psi == NULL)
        return -1;
    double h = 0.5 * dt;
    double J[3] = {hbar * hbar / (2.0 * mass * dx * dx), hbar * hbar / (2.0 * mass * dy * dy),
                   hbar * hbar / (2.0 * mass * dz * dz)};
    double eps0 = 2.0 * (J[0] + J[1] + J[2]);
    double sa[3], da[3];
    for (int a = 0; a < 3; ++a) block_coeffs(h, J[a], hbar, &sa[a], &da[a]);
    for (long long n = 0; n < steps; ++n) {
        for (int a = 0; a < 3; ++a) sweep3(nx, ny, nz, bc, a, 1, sa[a], da[a], psi);  /* O(h) */
        for (int a = 0; a < 3; ++a) sweep3(nx, ny, nz, bc, a, 0, sa[a], da[a], psi);  /* E(h) */
        potential_phase(nx, ny * nz, dt, eps0, hbar, V, psi);
        for (int a = 2; a >= 0; --a) sweep3(nx, ny, nz, bc, a, 0, sa[a], da[a], psi); /* E(h) */
        for (int a = 2; a >= 0; --a) sweep3(nx, ny, nz, bc, a, 1, sa[a], da[a], psi); /* O(h) */
    }
    return 0;
}

/* Norm and energy <psi|H|psi>/N on a (nz, ny, nx) mesh, six neighbours
 * (wrapping periodically, absent beyond closed walls); plane partial sums in
 * plane order. */
int tso_observables3(int nx, int ny, int nz, int bc, double dx, double dy, double dz,
                     double mass, double hbar, const double *V, const double *psi,
                     double *norm_out, double *energy_out) {
    if (!sides_ok(nx, ny, bc) || !sides_ok(nz, 2, bc) || !params_ok(dx, dy, mass, hbar) ||
        !(isfinite(dz) && dz > 0) || V == NULL || psi == NULL || norm_out == NULL ||
        energy_out == NULL)
        return -1;
    double J[3] = {hbar * hbar / (2.0 * mass * dx * dx), hbar * hbar / (2.0 * mass * dy * dy),
                   hbar * hbar / (2.0 * mass * dz * dz)};
    double eps0 = 2.0 * (J[0] + J[1] + J[2]);
    int n3[3] = {nx, ny, nz};
    double *pn = (double *)calloc((size_t)nz, sizeof(double));
    double *pe = (double *)calloc((size_t)nz, sizeof(double));
    if (!pn || !pe) {
        free(pn);
        free(pe);
        return -1;
    }
    int z;
#pragma omp parallel for schedule(static)
    for (z = 0; z < nz; ++z) {
        double sn = 0.0, se = 0.0;
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                int c[3] = {x, y, z};
                size_t l = ((size_t)z * ny + y) * nx + x;
                double pr = psi[2 * l], pi = psi[2 * l + 1];
                double hr = (V[l] + eps0) * pr, hi = (V[l] + eps0) * pi;
                for (int a = 0; a < 3; ++a)
                    for (int dir = -1; dir <= 1; dir += 2) {
                        int cc[3] = {c[0], c[1], c[2]};
                        cc[a] += dir;
                        if (cc[a] < 0 || cc[a] >= n3[a]) {
                            if (bc == TSO_BC_CLOSED) continue;
                            cc[a] = (cc[a] + n3[a]) % n3[a];
                        }
                        size_t m = ((size_t)cc[2] * ny + cc[1]) * nx + cc[0];
                        hr -= J[a] * psi[2 * m];
                        hi -= J[a] * psi[2 * m + 1];
                    }
                sn += pr * pr + pi * pi;
                se += pr * hr + pi * hi;
            }
        pn[z] = sn;
        pe[z] = se;
    }
    double n = 0.0, e = 0.0;
    for (z = 0; z < nz; ++z) {
        n += pn[z];
        e += pe[z];
    }
    free(pn);
    free(pe);
    *norm_out = n;
    *energy_out = (n > 0.0) ? e / n : 0.0;
    return 0;
}

/* Apply one single factor, for tests of the operator structure:
 *   which = 0: Kx(parity, tau)   1: Ky(parity, tau)   2: P(tau) */
int tso_apply_factor(int nx, int ny, int bc, double dx, double dy, double mass, double hbar,
                     int which, int parity, double tau, const double *V, double *psi) {
    if (!sides_ok(nx, ny, bc) || !params_ok(dx, dy, mass, hbar) || !isfinite(tau) ||
        psi == NULL || (parity != 0 && parity != 1))
        return -1;
    double s, d;
    if (which == 0) {
        block_coeffs(tau, hbar * hbar / (2.0 * mass * dx * dx), hbar, &s, &d);
        sweep_x(nx, ny, bc, parity, s, d, psi);
    } else if (which == 1) {
        block_coeffs(tau, hbar * hbar / (2.0 * mass * dy * dy), hbar, &s, &d);
        sweep_y(nx, ny, bc, parity, s, d, psi);
    } else if (which == 2) {
        if (V == NULL) return -1;
        double eps0 = hbar * hbar / (mass * dx * dx) + hbar * hbar / (mass * dy * dy);
        potential_phase(nx, ny, tau, eps0, hbar, V, psi);
    } else {
        return -1;
    }
    return 0;
}

/*
 * Norm N = sum_l |psi_l|^2 (Sec. 2, the norm conservation argument) and the
 * energy E = <psi|H|psi> / N of the lattice Hamiltonian
 *   (H psi)_l = eps_l psi_l - Jx (psi_{l+x} + psi_{l-x}) - Jy (psi_{l+y} + psi_{l-y}),
 * neighbours wrapping under periodic boundaries and absent at closed walls.
 * Row partial sums are added in row order, so the result does not depend on
 * the thread count.
 */
int tso_observables(int nx, int ny, int bc, double dx, double dy, double mass, double hbar,
                    const double *V, const double *psi, double *norm_out, double *energy_out) {
    if (!sides_ok(nx, ny, bc) || !params_ok(dx, dy, mass, hbar) || V == NULL || psi == NULL ||
        norm_out == NULL || energy_out == NULL)
        return -1;
    double Jx = hbar * hbar / (2.0 * mass * dx * dx);
    double Jy = hbar * hbar / (2.0 * mass * dy * dy);
    double eps0 = 2.0 * Jx + 2.0 * Jy;
    double *row_n = (double *)calloc((size_t)ny, sizeof(double));
    double *row_e = (double *)calloc((size_t)ny, sizeof(double));
    if (!row_n || !row_e) {
        free(row_n);
        free(row_e);
        return -1;
    }
    int y;
#pragma omp parallel for schedule(static)
    for (y = 0; y < ny; ++y) {
        double sn = 0.0, se = 0.0;
        for (int x = 0; x < nx; ++x) {
            size_t l = (size_t)y * nx + x;
            double pr = psi[2 * l], pi = psi[2 * l + 1];
            double hr = (V[l] + eps0) * pr, hi = (V[l] + eps0) * pi;
            int nbx[2] = {x + 1, x - 1}, nby[2] = {y + 1, y - 1};
            for (int k = 0; k < 2; ++k) {
                int xx = nbx[k];
                if (xx < 0 || xx >= nx) {
                    if (bc == TSO_BC_CLOSED) continue;
                    xx = (xx + nx) % nx;
                }
                size_t m = (size_t)y * nx + xx;
                hr -= Jx * psi[2 * m];
                hi -= Jx * psi[2 * m + 1];
            }
            for (int k = 0; k < 2; ++k) {
                int yy = nby[k];
                if (yy < 0 || yy >= ny) {
                    if (bc == TSO_BC_CLOSED) continue;
                    yy = (yy + ny) % ny;
                }
                size_t m = (size_t)yy * nx + x;
                hr -= Jy * psi[2 * m];
                hi -= Jy * psi[2 * m + 1];
            }
            sn += pr * pr + pi * pi;
            /* Re(conj(psi) * Hpsi) */
            se += pr * hr + pi * hi;
        }
        row_n[y] = sn;
        row_e[y] = se;
    }
    double n = 0.0, e = 0.0;
    for (y = 0; y < ny; ++y) {
        n += row_n[y];
        e += row_e[y];
    }
    free(row_n);
    free(row_e);
    *norm_out = n;
    *energy_out = (n > 0.0) ? e / n : 0.0;
    return 0;
}
