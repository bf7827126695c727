/*
 * moto_oracle.c -- plain FP64 CPU oracle for the bilayer minimum-mode kernel
 * (Xu & Delin, "A general optimization framework for mapping local
 * transition-state networks", arXiv 2509.26269).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant generator
 * with the HIP library: every quantity is re-derived here from the paper.
 *
 * Everything is written the slow, obvious way: single-threaded loops over
 * ordered site pairs, FP64 throughout, no blocking or fusion.
 *
 * Conventions (readings of the paper, see the design notes):
 *   - periodic rhombic Lx x Ly triangular lattice, a1 = (1,0), a2 = (1/2, sqrt3/2),
 *     site s = x + Lx*y, nearest-neighbour distance 1;
 *   - spins stored SoA: m[0*N + s] = mx, m[1*N + s] = my, m[2*N + s] = mz;
 *   - the energy is the Methods-section spin Hamiltonian (Eq. "param-hamiltonian")
 *     with the sums read literally as sums over ordered pairs i != j, i.e. as
 *     sum_i sum_{delta} over every lattice offset delta of a shell;
 *   - mu_i = 1, K uniform with easy axis e_z, B a vector;
 *   - DMI vector of offset delta in shell s: D_delta = D_s (z x dhat).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_SHELLS 36
#define ORC_MAX_OFFSETS 512
#define ORC_SEARCH_R 12
#define ORC_MAX_GEN_SHELLS 64

typedef struct {
    int32_t Lx, Ly, n_shells;
    int32_t pad_;
    double J[ORC_MAX_SHELLS];
    double D[ORC_MAX_SHELLS];
    double K;
    double B[3];
} orc_ham;

/* ------------------------------------------------------------------ */
/* Lattice shells: every lattice vector dx*a1 + dy*a2 sorted by length.
 * |dx a1 + dy a2|^2 = dx^2 + dx*dy + dy^2 exactly (an integer).
 * Shell s collects all offsets at the s-th smallest nonzero distance.
 * Returns the number of offsets written (or -1 if cap is too small). */
int orc_shells(int n_shells, int *dx_out, int *dy_out, int *shell_out, int cap)
{
    int d2_list[(2 * ORC_SEARCH_R + 1) * (2 * ORC_SEARCH_R + 1)];
    int n_d2 = 0;
    if (n_shells < 0 || n_shells > ORC_MAX_GEN_SHELLS) return -1;
    /* distinct squared lengths, ascending (insertion into a sorted list) */
    for (int dy = -ORC_SEARCH_R; dy <= ORC_SEARCH_R; ++dy)
        for (int dx = -ORC_SEARCH_R; dx <= ORC_SEARCH_R; ++dx) {
            int d2 = dx * dx + dx * dy + dy * dy;
            if (d2 == 0) continue;
            int seen = 0;
            for (int k = 0; k < n_d2; ++k) if (d2_list[k] == d2) { seen = 1; break; }
            if (seen) continue;
            int k = n_d2++;
            while (k > 0 && d2_list[k - 1] > d2) { d2_list[k] = d2_list[k - 1]; --k; }
            d2_list[k] = d2;
        }
    int n = 0;
    for (int s = 0; s < n_shells; ++s)
        for (int dy = -ORC_SEARCH_R; dy <= ORC_SEARCH_R; ++dy)
            for (int dx = -ORC_SEARCH_R; dx <= ORC_SEARCH_R; ++dx)
                if (dx * dx + dx * dy + dy * dy == d2_list[s]) {
                    if (n >= cap) return -1;
                    dx_out[n] = dx; dy_out[n] = dy; shell_out[n] = s; ++n;
                }
    return n;
}

/* One ordered neighbour term of the Hamiltonian: offset (dx,dy), exchange J,
 * DMI vector Dv. */
typedef struct { int dx, dy, shell; double J; double Dv[3]; } orc_term;

static int build_terms(const orc_ham *h, orc_term *t)
{
    int dx[ORC_MAX_OFFSETS], dy[ORC_MAX_OFFSETS], sh[ORC_MAX_OFFSETS];
    int n = orc_shells(h->n_shells, dx, dy, sh, ORC_MAX_OFFSETS);
    const double s3 = sqrt(3.0);
    for (int k = 0; k < n; ++k) {
        double rx = dx[k] + 0.5 * dy[k];
        double ry = 0.5 * s3 * dy[k];
        double r = sqrt(rx * rx + ry * ry);
        double ux = rx / r, uy = ry / r;
        t[k].dx = dx[k]; t[k].dy = dy[k]; t[k].shell = sh[k];
        t[k].J = h->J[sh[k]];
        /* D_delta = D_s * (z x dhat) = D_s * (-dhat_y, dhat_x, 0) */
        t[k].Dv[0] = -h->D[sh[k]] * uy;
        t[k].Dv[1] = h->D[sh[k]] * ux;
        t[k].Dv[2] = 0.0;
    }
    return n;
}

static inline int site_add(int Lx, int Ly, int s, int dx, int dy)
{
    int x = s % Lx, y = s / Lx;
    x = ((x + dx) % Lx + Lx) % Lx;
    y = ((y + dy) % Ly + Ly) % Ly;
    return x + Lx * y;
}

static inline void cross3(const double *a, const double *b, double *o)
{
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}

static inline void get3(const double *v, int N, int s, double *o)
{
    o[0] = v[s]; o[1] = v[N + s]; o[2] = v[2 * N + s];
}

/* ------------------------------------------------------------------ */
/* Energy, term by term (Methods, Eq. "param-hamiltonian"):
 *   terms[0] = -sum_i sum_delta J_delta m_i . m_{i+delta}
 *   terms[1] = -sum_i sum_delta D_delta . (m_i x m_{i+delta})
 *   terms[2] = -sum_i B . m_i
 *   terms[3] = -K sum_i (m_i . e_z)^2
 *   terms[4] = total
 * Also, if dtheta != NULL, the partial derivatives of E with respect to the
 * Hamiltonian parameters theta = (J_0..J_{ns-1}, D_0..D_{ns-1}, K, Bx, By, Bz):
 * E is linear in theta, so each partial is the sum multiplying it. */
void orc_energy(const orc_ham *h, const double *m, double *terms, double *dtheta)
{
    orc_term t[ORC_MAX_OFFSETS];
    int nt = build_terms(h, t);
    int N = h->Lx * h->Ly, ns = h->n_shells;
    double e_ex = 0, e_dmi = 0, e_z = 0, e_k = 0;
    double dJ[ORC_MAX_SHELLS] = {0}, dD[ORC_MAX_SHELLS] = {0};
    double dK = 0, dB[3] = {0, 0, 0};
    for (int i = 0; i < N; ++i) {
        double mi[3];
        get3(m, N, i, mi);
        for (int k = 0; k < nt; ++k) {
            int j = site_add(h->Lx, h->Ly, i, t[k].dx, t[k].dy);
            double mj[3], x[3];
            get3(m, N, j, mj);
            double dot = mi[0] * mj[0] + mi[1] * mj[1] + mi[2] * mj[2];
            cross3(mi, mj, x);
            double r = sqrt((t[k].dx + 0.5 * t[k].dy) * (t[k].dx + 0.5 * t[k].dy)
                            + 0.75 * t[k].dy * t[k].dy);
            double zxd[3] = {-(0.5 * sqrt(3.0) * t[k].dy) / r, (t[k].dx + 0.5 * t[k].dy) / r, 0.0};
            double dmi_unit = zxd[0] * x[0] + zxd[1] * x[1] + zxd[2] * x[2];
            e_ex += -t[k].J * dot;
            e_dmi += -(t[k].Dv[0] * x[0] + t[k].Dv[1] * x[1] + t[k].Dv[2] * x[2]);
            dJ[t[k].shell] += -dot;
            dD[t[k].shell] += -dmi_unit;
        }
        e_z += -(h->B[0] * mi[0] + h->B[1] * mi[1] + h->B[2] * mi[2]);
        e_k += -h->K * mi[2] * mi[2];
        dK += -mi[2] * mi[2];
        dB[0] += -mi[0]; dB[1] += -mi[1]; dB[2] += -mi[2];
    }
    terms[0] = e_ex; terms[1] = e_dmi; terms[2] = e_z; terms[3] = e_k;
    terms[4] = e_ex + e_dmi + e_z + e_k;
    if (dtheta) {
        for (int s = 0; s < ns; ++s) { dtheta[s] = dJ[s]; dtheta[ns + s] = dD[s]; }
        dtheta[2 * ns] = dK;
        dtheta[2 * ns + 1] = dB[0]; dtheta[2 * ns + 2] = dB[1]; dtheta[2 * ns + 3] = dB[2];
    }
}

/* Euclidean gradient g = dE/dm, by differentiating every ordered pair term
 * with respect to both of its spins and scattering the result:
 *   -J m_i.m_j        -> g_i += -J m_j,          g_j += -J m_i
 *   -D.(m_i x m_j)    -> g_i += -(m_j x D),      g_j += -(D x m_i)
 *   -B.m_i            -> g_i += -B
 *   -K m_iz^2         -> g_iz += -2 K m_iz                                 */
void orc_gradient(const orc_ham *h, const double *m, double *g)
{
    orc_term t[ORC_MAX_OFFSETS];
    int nt = build_terms(h, t);
    int N = h->Lx * h->Ly;
    memset(g, 0, sizeof(double) * 3 * (size_t)N);
    for (int i = 0; i < N; ++i) {
        double mi[3];
        get3(m, N, i, mi);
        for (int k = 0; k < nt; ++k) {
            int j = site_add(h->Lx, h->Ly, i, t[k].dx, t[k].dy);
            double mj[3], a[3], b[3];
            get3(m, N, j, mj);
            cross3(mj, t[k].Dv, a);
            cross3(t[k].Dv, mi, b);
            for (int c = 0; c < 3; ++c) {
                g[c * N + i] += -t[k].J * mj[c] - a[c];
                g[c * N + j] += -t[k].J * mi[c] - b[c];
            }
        }
        for (int c = 0; c < 3; ++c) g[c * N + i] += -h->B[c];
        g[2 * N + i] += -2.0 * h->K * mi[2];
    }
}

/* Euclidean Hessian-vector product out = A v.  E is quadratic plus linear
 * in m, so A is the constant bilinear part of the gradient (the same scatter
 * rules as orc_gradient without the Zeeman term).                          */
void orc_apply_A(const orc_ham *h, const double *v, double *out)
{
    orc_term t[ORC_MAX_OFFSETS];
    int nt = build_terms(h, t);
    int N = h->Lx * h->Ly;
    memset(out, 0, sizeof(double) * 3 * (size_t)N);
    for (int i = 0; i < N; ++i) {
        double vi[3];
        get3(v, N, i, vi);
        for (int k = 0; k < nt; ++k) {
            int j = site_add(h->Lx, h->Ly, i, t[k].dx, t[k].dy);
            double vj[3], a[3], b[3];
            get3(v, N, j, vj);
            cross3(vj, t[k].Dv, a);
            cross3(t[k].Dv, vi, b);
            for (int c = 0; c < 3; ++c) {
                out[c * N + i] += -t[k].J * vj[c] - a[c];
                out[c * N + j] += -t[k].J * vi[c] - b[c];
            }
        }
        out[2 * N + i] += -2.0 * h->K * vi[2];
    }
}

/* Weingarten scalar c_i = m_i . g_i and tangent force F_i = -(I - m_i m_i^T) g_i
 * (Methods: forces are the negative gradient, tangent-projected for spins). */
void orc_force(int N, const double *m, const double *g, double *c, double *F)
{
    for (int i = 0; i < N; ++i) {
        double ci = m[i] * g[i] + m[N + i] * g[N + i] + m[2 * N + i] * g[2 * N + i];
        if (c) c[i] = ci;
        if (F)
            for (int k = 0; k < 3; ++k) F[k * N + i] = -(g[k * N + i] - ci * m[k * N + i]);
    }
}

/* Riemannian (tangent) Hessian-vector product on the product of unit spheres:
 *   (H v)_i = P_i (A v)_i - c_i v_i,     P_i = I - m_i m_i^T,
 * for tangent v (v_i . m_i = 0).  With a mask (nonzero = active site) this is
 * the principal submatrix on the active set: w = M H (M v).  mask may be NULL. */
void orc_tangent_hvp(const orc_ham *h, const double *m, const double *c,
                     const uint8_t *mask, const double *v, double *w)
{
    int N = h->Lx * h->Ly;
    double *vm = (double *)malloc(sizeof(double) * 3 * (size_t)N);
    double *Av = (double *)malloc(sizeof(double) * 3 * (size_t)N);
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < N; ++i)
            vm[k * N + i] = (mask && !mask[i]) ? 0.0 : v[k * N + i];
    orc_apply_A(h, vm, Av);
    for (int i = 0; i < N; ++i) {
        double mi[3], ti[3];
        get3(m, N, i, mi);
        get3(Av, N, i, ti);
        double mt = mi[0] * ti[0] + mi[1] * ti[1] + mi[2] * ti[2];
        for (int k = 0; k < 3; ++k) {
            double val = ti[k] - mt * mi[k] - c[i] * vm[k * N + i];
            w[k * N + i] = (mask && !mask[i]) ? 0.0 : val;
        }
    }
    free(vm);
    free(Av);
}

/* Euclidean Hessian assembled entry by entry from the ENERGY alone, by the
 * four-point mixed central difference with step h_fd.  E is a polynomial of
 * degree two in m, so the difference is exact up to rounding for any step;
 * H must hold (3N)^2 doubles, row-major, index a = comp*N + site.  Tiny
 * lattices only. */
void orc_dense_hessian_fd(const orc_ham *h, const double *m, double h_fd, double *H)
{
    int N = h->Lx * h->Ly, n = 3 * N;
    double *x = (double *)malloc(sizeof(double) * (size_t)n);
    double terms[5];
    for (int a = 0; a < n; ++a)
        for (int b = 0; b < n; ++b) {
            double e[4];
            const int sa[4] = {+1, +1, -1, -1}, sb[4] = {+1, -1, +1, -1};
            for (int q = 0; q < 4; ++q) {
                memcpy(x, m, sizeof(double) * (size_t)n);
                x[a] += sa[q] * h_fd;
                x[b] += sb[q] * h_fd;
                orc_energy(h, x, terms, NULL);
                e[q] = terms[4];
            }
            H[(size_t)a * n + b] = (e[0] - e[1] - e[2] + e[3]) / (4.0 * h_fd * h_fd);
        }
    free(x);
}

/* Cyclic Jacobi eigenvalue algorithm for a dense symmetric matrix
 * (Golub & Van Loan, Matrix Computations, the cyclic-by-row Jacobi method
 * with the symmetric 2x2 Schur rotation).  A (n x n, row-major) is
 * overwritten; evals[n] unsorted; V (n x n, row-major) holds eigenvectors in
 * its COLUMNS.  Returns the number of sweeps used, or -1 if not converged. */
int orc_jacobi_eig(int n, double *A, double *evals, double *V, double tol, int max_sweeps)
{
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < n; ++j) V[(size_t)i * n + j] = (i == j) ? 1.0 : 0.0;
    double fro = 0.0;
    for (size_t q = 0; q < (size_t)n * n; ++q) fro += A[q] * A[q];
    fro = sqrt(fro);
    int sweep;
    for (sweep = 0; sweep < max_sweeps; ++sweep) {
        double off = 0.0;
        for (int p = 0; p < n; ++p)
            for (int q = 0; q < n; ++q)
                if (p != q) off += A[(size_t)p * n + q] * A[(size_t)p * n + q];
        if (sqrt(off) <= tol * fro) break;
        for (int p = 0; p < n - 1; ++p)
            for (int q = p + 1; q < n; ++q) {
                double apq = A[(size_t)p * n + q];
                if (apq == 0.0) continue;
                double app = A[(size_t)p * n + p], aqq = A[(size_t)q * n + q];
                double tau = (aqq - app) / (2.0 * apq);
                double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                double cs = 1.0 / sqrt(1.0 + t * t), sn = t * cs;
                /* A <- J^T A J with J the rotation in the (p,q) plane */
                for (int k = 0; k < n; ++k) {
                    double akp = A[(size_t)k * n + p], akq = A[(size_t)k * n + q];
                    A[(size_t)k * n + p] = cs * akp - sn * akq;
                    A[(size_t)k * n + q] = sn * akp + cs * akq;
                }
                for (int k = 0; k < n; ++k) {
                    double apk = A[(size_t)p * n + k], aqk = A[(size_t)q * n + k];
                    A[(size_t)p * n + k] = cs * apk - sn * aqk;
                    A[(size_t)q * n + k] = sn * apk + cs * aqk;
                }
                for (int k = 0; k < n; ++k) {
                    double vkp = V[(size_t)k * n + p], vkq = V[(size_t)k * n + q];
                    V[(size_t)k * n + p] = cs * vkp - sn * vkq;
                    V[(size_t)k * n + q] = sn * vkp + cs * vkq;
                }
            }
    }
    for (int i = 0; i < n; ++i) evals[i] = A[(size_t)i * n + i];
    return sweep < max_sweeps ? sweep : -1;
}

/* Berg-Luescher lattice topological charge (Berg & Luescher 1981):
 *   Q = -(1/4pi) sum over counter-clockwise triangles of the signed solid
 *       angle 2 atan2(m_i.(m_j x m_k), 1 + m_i.m_j + m_j.m_k + m_k.m_i).
 * Two triangles per rhombic cell: (x,y),(x+1,y),(x,y+1) and
 * (x+1,y),(x+1,y+1),(x,y+1).  The leading minus makes a core-down Neel
 * skyrmion in a +z background count +1.                                    */
double orc_topological_charge(int Lx, int Ly, const double *m)
{
    int N = Lx * Ly;
    double q = 0.0;
    for (int y = 0; y < Ly; ++y)
        for (int x = 0; x < Lx; ++x) {
            int s00 = x + Lx * y;
            int s10 = (x + 1) % Lx + Lx * y;
            int s01 = x + Lx * ((y + 1) % Ly);
            int s11 = (x + 1) % Lx + Lx * ((y + 1) % Ly);
            int tri[2][3] = {{s00, s10, s01}, {s10, s11, s01}};
            for (int t = 0; t < 2; ++t) {
                double a[3], b[3], c[3], bc[3];
                get3(m, N, tri[t][0], a);
                get3(m, N, tri[t][1], b);
                get3(m, N, tri[t][2], c);
                cross3(b, c, bc);
                double num = a[0] * bc[0] + a[1] * bc[1] + a[2] * bc[2];
                double den = 1.0 + (a[0] * b[0] + a[1] * b[1] + a[2] * b[2])
                           + (b[0] * c[0] + b[1] * c[1] + b[2] * c[2])
                           + (c[0] * a[0] + c[1] * a[1] + c[2] * a[2]);
                q += 2.0 * atan2(num, den);
            }
        }
    return -q / (4.0 * M_PI);
}
