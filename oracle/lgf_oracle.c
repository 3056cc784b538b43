/*
 * lgf_oracle.c -- plain FP64 CPU oracle for checkerboard SU(3) Landau gauge
 * fixing by overrelaxation (OR) and stochastic relaxation (SR), following
 * M. Schroeck and H. Vogt, "Gauge fixing in lattice QCD with multi-GPUs"
 * (arXiv:1305.3440).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness reference for the
 * HIP library.  Only the test suite, the package smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no code, header,
 * table or constant with the HIP path; its random numbers come from its own
 * Philox4x32-10, written from the published definition (Salmon, Moraes,
 * Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11).
 *
 * Everything is double precision, written for a reader to check against the
 * paper: no blocking, no fusion, no reordering beyond what the paper states.
 * The only parallelism is over the sites of one parity (OpenMP), which the
 * paper states are independent (Sec. 3, checkerboard decomposition); every
 * reduction is summed serially in site order, so results are deterministic.
 *
 * Equation numbers (1)-(9) count the displayed equations of the paper in
 * order of appearance: (2) functional F, (3) gauge transformation, (4) Delta,
 * (5) theta, (6) local form of F, (7) f(x), (8) K(x), (9) SU(2) maximum.
 *
 * Readings where the paper is silent (each one also has a pin in the tests):
 *  - A_mu(x) = [(U - U^dag)/(2i)]_traceless, lattice spacing and coupling 1.
 *  - After a site update the links are transformed in place, so the neighbour
 *    g's in Eq. (8) are already absorbed: K = sum_mu U_mu(x) + U_mu(x-mu)^dag.
 *  - Cabibbo-Marinari subgroups in the order (0,1), (0,2), (1,2), one pass per
 *    site update; OR and SR act on each SU(2) subgroup element.
 *  - First-order OR: r_w = N[(1 - w) 1 + w r], N = normalise the quaternion.
 *  - SR: per subgroup, r -> r^2 when a Philox word is below floor(p 2^32).
 *  - A degenerate block (zero quaternion projection) leaves the site alone.
 *  - Parity of a site is (t+z+y+x) mod 2; parity 0 is swept first.
 *
 * Lattice: dims = (Lt, Lz, Ly, Lx), mu = 0 is t, 1 z, 2 y, 3 x; the site index
 * is s = ((t*Lz + z)*Ly + y)*Lx + x; periodic boundaries.  The link array is
 * double[V][4][3][3][2] (site, mu, row, column, re/im): 72 doubles per site.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;
typedef struct { cplx m[3][3]; } mat3;

/* ------------------------------------------------------------------------ */
/* 3x3 complex matrices                                                      */
/* ------------------------------------------------------------------------ */

static mat3 mat_load(const double *p)
{
    mat3 a;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            a.m[i][j] = p[2 * (3 * i + j)] + I * p[2 * (3 * i + j) + 1];
    return a;
}

static void mat_store(const mat3 *a, double *p)
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            p[2 * (3 * i + j)] = creal(a->m[i][j]);
            p[2 * (3 * i + j) + 1] = cimag(a->m[i][j]);
        }
}

static mat3 mat_identity(void)
{
    mat3 a;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            a.m[i][j] = (i == j) ? 1.0 : 0.0;
    return a;
}

static mat3 mat_zero(void)
{
    mat3 a;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            a.m[i][j] = 0.0;
    return a;
}

static mat3 mat_mul(const mat3 *a, const mat3 *b)
{
    mat3 c;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            cplx s = 0.0;
            for (int k = 0; k < 3; ++k)
                s += a->m[i][k] * b->m[k][j];
            c.m[i][j] = s;
        }
    return c;
}

static mat3 mat_dag(const mat3 *a)
{
    mat3 c;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            c.m[i][j] = conj(a->m[j][i]);
    return c;
}

static mat3 mat_add(const mat3 *a, const mat3 *b)
{
    mat3 c;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            c.m[i][j] = a->m[i][j] + b->m[i][j];
    return c;
}

static mat3 mat_sub(const mat3 *a, const mat3 *b)
{
    mat3 c;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            c.m[i][j] = a->m[i][j] - b->m[i][j];
    return c;
}

static mat3 mat_scale(const mat3 *a, cplx s)
{
    mat3 c;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            c.m[i][j] = s * a->m[i][j];
    return c;
}

static cplx mat_trace(const mat3 *a)
{
    return a->m[0][0] + a->m[1][1] + a->m[2][2];
}

static cplx mat_det(const mat3 *a)
{
    const cplx (*m)[3] = a->m;
    return m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1])
         - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0])
         + m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
}

static double mat_norm2(const mat3 *a) /* squared Frobenius norm */
{
    double s = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            s += creal(a->m[i][j]) * creal(a->m[i][j])
               + cimag(a->m[i][j]) * cimag(a->m[i][j]);
    return s;
}

/* Project onto SU(3): normalise row 0, Gram-Schmidt row 1 against it, and
 * take row 2 = conj(row0 x row1), the cofactor form of the last row of a
 * unitary matrix with determinant one. */
static mat3 mat_reunitarize(const mat3 *a)
{
    cplx u[3], v[3];
    double nu = 0.0;
    for (int k = 0; k < 3; ++k) nu += creal(a->m[0][k] * conj(a->m[0][k]));
    nu = sqrt(nu);
    for (int k = 0; k < 3; ++k) u[k] = a->m[0][k] / nu;
    cplx uv = 0.0; /* <u, r1> = sum_k conj(u_k) r1_k */
    for (int k = 0; k < 3; ++k) uv += conj(u[k]) * a->m[1][k];
    for (int k = 0; k < 3; ++k) v[k] = a->m[1][k] - uv * u[k];
    double nv = 0.0;
    for (int k = 0; k < 3; ++k) nv += creal(v[k] * conj(v[k]));
    nv = sqrt(nv);
    for (int k = 0; k < 3; ++k) v[k] /= nv;
    mat3 r;
    for (int k = 0; k < 3; ++k) { r.m[0][k] = u[k]; r.m[1][k] = v[k]; }
    r.m[2][0] = conj(u[1] * v[2] - u[2] * v[1]);
    r.m[2][1] = conj(u[2] * v[0] - u[0] * v[2]);
    r.m[2][2] = conj(u[0] * v[1] - u[1] * v[0]);
    return r;
}

/* ------------------------------------------------------------------------ */
/* Lattice geometry                                                          */
/* ------------------------------------------------------------------------ */

typedef struct { int L[4]; int64_t V; } lattice;

static lattice make_lattice(const int dims[4])
{
    lattice lat;
    lat.V = 1;
    for (int d = 0; d < 4; ++d) { lat.L[d] = dims[d]; lat.V *= dims[d]; }
    return lat;
}

static void site_coords(const lattice *lat, int64_t s, int c[4])
{
    for (int d = 3; d >= 0; --d) { c[d] = (int)(s % lat->L[d]); s /= lat->L[d]; }
}

static int64_t site_index(const lattice *lat, const int c[4])
{
    int64_t s = 0;
    for (int d = 0; d < 4; ++d) s = s * lat->L[d] + c[d];
    return s;
}

/* neighbour of site s one step (step = +1 or -1) in direction mu, periodic */
static int64_t site_neighbor(const lattice *lat, int64_t s, int mu, int step)
{
    int c[4];
    site_coords(lat, s, c);
    c[mu] = (c[mu] + step + lat->L[mu]) % lat->L[mu];
    return site_index(lat, c);
}

static int site_parity(const lattice *lat, int64_t s)
{
    int c[4];
    site_coords(lat, s, c);
    return (c[0] + c[1] + c[2] + c[3]) & 1;
}

static double *link_ptr(double *U, int64_t s, int mu) { return U + (s * 4 + mu) * 18; }
static const double *link_cptr(const double *U, int64_t s, int mu) { return U + (s * 4 + mu) * 18; }

int64_t orc_volume(const int dims[4]) { return make_lattice(dims).V; }

int64_t orc_neighbor(const int dims[4], int64_t s, int mu, int step)
{
    lattice lat = make_lattice(dims);
    return site_neighbor(&lat, s, mu, step);
}

int orc_parity(const int dims[4], int64_t s)
{
    lattice lat = make_lattice(dims);
    return site_parity(&lat, s);
}

/* Indices (s*4 + mu) of the 8 links a site update touches: the 4 forward
 * links U_mu(x) and the 4 backward links U_mu(x - mu). */
void orc_site_links(const int dims[4], int64_t s, int64_t idx[8])
{
    lattice lat = make_lattice(dims);
    for (int mu = 0; mu < 4; ++mu) {
        idx[mu] = s * 4 + mu;
        idx[4 + mu] = site_neighbor(&lat, s, mu, -1) * 4 + mu;
    }
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon et al., SC'11): ten rounds of the Philox S-box on a   */
/* 128-bit counter with a 64-bit key bumped by the Weyl constants each round. */
/* ------------------------------------------------------------------------ */

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        if (round > 0) { k0 += W0; k1 += W1; }
        uint64_t p0 = (uint64_t)M0 * x0;
        uint64_t p1 = (uint64_t)M1 * x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        x0 = y0; x1 = lo1; x2 = y2; x3 = lo0;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

static void philox_seeded(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                          uint32_t c3, uint32_t out[4])
{
    const uint32_t ctr[4] = {c0, c1, c2, c3};
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    orc_philox4x32_10(ctr, key, out);
}

/* Four standard normals from one Philox call: Box-Muller on the word pairs
 * (0,1) and (2,3), with uniforms u = (w + 1/2) 2^-32 in (0,1). */
static void normals4(uint64_t seed, uint32_t c0, uint32_t c1, uint32_t c2,
                     uint32_t c3, double n[4])
{
    uint32_t w[4];
    philox_seeded(seed, c0, c1, c2, c3, w);
    const double two_m32 = 1.0 / 4294967296.0;
    for (int pair = 0; pair < 2; ++pair) {
        double u1 = ((double)w[2 * pair] + 0.5) * two_m32;
        double u2 = ((double)w[2 * pair + 1] + 0.5) * two_m32;
        double r = sqrt(-2.0 * log(u1));
        n[2 * pair] = r * cos(2.0 * M_PI * u2);
        n[2 * pair + 1] = r * sin(2.0 * M_PI * u2);
    }
}

void orc_normals4(uint64_t seed, const uint32_t ctr[4], double n[4])
{
    normals4(seed, ctr[0], ctr[1], ctr[2], ctr[3], n);
}

/* ------------------------------------------------------------------------ */
/* Synthetic gauge fields: U = exp(i eps sum_j a_j lambda_j) with normal a_j,  */
/* then a Haar-random gauge transformation (Eq. (3)).                         */
/* ------------------------------------------------------------------------ */

/* H = sum_j a_j lambda_j with the Gell-Mann matrices (tr lambda_a lambda_b =
 * 2 delta_ab). */
static mat3 gellmann_combination(const double a[8])
{
    const double s3 = 1.0 / sqrt(3.0);
    mat3 H;
    H.m[0][0] = a[2] + a[7] * s3;
    H.m[1][1] = -a[2] + a[7] * s3;
    H.m[2][2] = -2.0 * a[7] * s3;
    H.m[0][1] = a[0] - I * a[1];
    H.m[1][0] = a[0] + I * a[1];
    H.m[0][2] = a[3] - I * a[4];
    H.m[2][0] = a[3] + I * a[4];
    H.m[1][2] = a[5] - I * a[6];
    H.m[2][1] = a[5] + I * a[6];
    return H;
}

/* exp(X) by scaling and squaring: halve X until its Frobenius norm is below
 * 1/2, sum the Taylor series to order 16, square back. */
static mat3 mat_exp(const mat3 *X)
{
    int k = 0;
    double nrm = sqrt(mat_norm2(X));
    while (nrm / ldexp(1.0, k) >= 0.5) ++k;
    mat3 Y = mat_scale(X, ldexp(1.0, -k));
    mat3 S = mat_identity(), term = mat_identity();
    for (int n = 1; n <= 16; ++n) {
        mat3 t = mat_mul(&term, &Y);
        term = mat_scale(&t, 1.0 / n);
        S = mat_add(&S, &term);
    }
    for (int i = 0; i < k; ++i) S = mat_mul(&S, &S);
    return S;
}

/* exp(i eps H(a)), then projected onto SU(3) */
void orc_su3_exp_iH(const double a[8], double eps, double out[18])
{
    mat3 H = gellmann_combination(a);
    mat3 X = mat_scale(&H, I * eps);
    mat3 E = mat_exp(&X);
    mat3 R = mat_reunitarize(&E);
    mat_store(&R, out);
}

/* Haar-random SU(3) element for site s: a complex Ginibre matrix (entries
 * (n + i n')/sqrt(2) from 18 normals), orthonormalised column by column (QR
 * with a positive real diagonal of R, which gives Haar measure on U(3)), then
 * divided by the principal cube root of its determinant. */
void orc_haar_su3(uint64_t seed, int64_t s, double out[18])
{
    double n[20];
    for (int call = 0; call < 5; ++call)
        normals4(seed, (uint32_t)s, 0u, (uint32_t)call, 2u, n + 4 * call);
    mat3 Z;
    const double r2 = 1.0 / sqrt(2.0);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            Z.m[i][j] = (n[2 * (3 * i + j)] + I * n[2 * (3 * i + j) + 1]) * r2;
    mat3 Q;
    for (int j = 0; j < 3; ++j) {
        cplx v[3];
        for (int i = 0; i < 3; ++i) v[i] = Z.m[i][j];
        for (int k = 0; k < j; ++k) {
            cplx proj = 0.0;
            for (int i = 0; i < 3; ++i) proj += conj(Q.m[i][k]) * v[i];
            for (int i = 0; i < 3; ++i) v[i] -= proj * Q.m[i][k];
        }
        double nv = 0.0;
        for (int i = 0; i < 3; ++i) nv += creal(v[i] * conj(v[i]));
        nv = sqrt(nv);
        for (int i = 0; i < 3; ++i) Q.m[i][j] = v[i] / nv;
    }
    double phi = carg(mat_det(&Q));
    mat3 g = mat_scale(&Q, cexp(-I * phi / 3.0));
    mat_store(&g, out);
}

/* The generated link U_mu(s) before any gauge transformation. */
static mat3 raw_link(uint64_t seed, double eps, int64_t s, int mu)
{
    double a[8];
    normals4(seed, (uint32_t)s, (uint32_t)mu, 0u, 1u, a);
    normals4(seed, (uint32_t)s, (uint32_t)mu, 1u, 1u, a + 4);
    double u[18];
    orc_su3_exp_iH(a, eps, u);
    return mat_load(u);
}

/* One link of the synthetic field: raw link, optionally gauge transformed by
 * the Haar field, g(x) U_mu(x) g(x+mu)^dag (Eq. (3)).  Each link depends only
 * on (seed, site, mu), so any single link can be generated on its own. */
void orc_generated_link(const int dims[4], uint64_t seed, double eps, int haar,
                        int64_t s, int mu, double out[18])
{
    lattice lat = make_lattice(dims);
    mat3 U = raw_link(seed, eps, s, mu);
    if (haar) {
        double gx[18], gy[18];
        orc_haar_su3(seed, s, gx);
        orc_haar_su3(seed, site_neighbor(&lat, s, mu, +1), gy);
        mat3 G1 = mat_load(gx), G2 = mat_load(gy);
        mat3 G2d = mat_dag(&G2);
        mat3 t = mat_mul(&G1, &U);
        U = mat_mul(&t, &G2d);
    }
    mat_store(&U, out);
}

void orc_generate_links(const int dims[4], uint64_t seed, double eps, int haar, double *U)
{
    lattice lat = make_lattice(dims);
    #pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < lat.V; ++s)
        for (int mu = 0; mu < 4; ++mu)
            orc_generated_link(dims, seed, eps, haar, s, mu, link_ptr(U, s, mu));
}

/* U_mu(x) <- g(x) U_mu(x) g(x+mu)^dag for a gauge field g[V][3][3][2], Eq. (3) */
void orc_gauge_transform(const int dims[4], double *U, const double *g)
{
    lattice lat = make_lattice(dims);
    #pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < lat.V; ++s) {
        mat3 gx = mat_load(g + 18 * s);
        for (int mu = 0; mu < 4; ++mu) {
            mat3 gy = mat_load(g + 18 * site_neighbor(&lat, s, mu, +1));
            mat3 gyd = mat_dag(&gy);
            mat3 u = mat_load(link_ptr(U, s, mu));
            mat3 t = mat_mul(&gx, &u);
            mat3 r = mat_mul(&t, &gyd);
            mat_store(&r, link_ptr(U, s, mu));
        }
    }
}

/* ------------------------------------------------------------------------ */
/* The relaxation step (Sec. 3)                                               */
/* ------------------------------------------------------------------------ */

/* One SU(2) subgroup step (Eq. (9) with Sec. 3.1 and 3.2).
 * w = {Re w00, Im w00, Re w01, Im w01, Re w10, Im w10, Re w11, Im w11} is the
 * 2x2 block of W = G K on the subgroup's rows and columns.  Writing a
 * quaternion a as the matrix s(a) = [[a0 + i a3, a2 + i a1], [-a2 + i a1,
 * a0 - i a3]], Re tr[s(b) w] = 2 (b0 a0 - b.a) where a is the quaternion part
 * of w; over unit b this is largest at b = (a0, -a)/|a| (value 2|a|), which is
 * the SU(2) solution K^dag / sqrt(det K^dag) of Eq. (9).
 * OR (Sec. 3.1): r = N[(1 - omega) + omega b], the first-order form of b^omega.
 * SR (Sec. 3.2, take_square != 0): r = b^2.
 * A zero projection (|a| = 0) returns the identity.  r = (r0, r1, r2, r3). */
void orc_su2_step(const double w[8], double omega, int take_square, double r[4])
{
    double a0 = 0.5 * (w[0] + w[6]);
    double a3 = 0.5 * (w[1] - w[7]);
    double a1 = 0.5 * (w[3] + w[5]);
    double a2 = 0.5 * (w[2] - w[4]);
    double na = sqrt(a0 * a0 + a1 * a1 + a2 * a2 + a3 * a3);
    if (na == 0.0) { r[0] = 1.0; r[1] = r[2] = r[3] = 0.0; return; }
    double b0 = a0 / na, b1 = -a1 / na, b2 = -a2 / na, b3 = -a3 / na;
    if (take_square) {
        r[0] = b0 * b0 - (b1 * b1 + b2 * b2 + b3 * b3);
        r[1] = 2.0 * b0 * b1;
        r[2] = 2.0 * b0 * b2;
        r[3] = 2.0 * b0 * b3;
    } else {
        double c0 = (1.0 - omega) + omega * b0;
        double c1 = omega * b1, c2 = omega * b2, c3 = omega * b3;
        double nc = sqrt(c0 * c0 + c1 * c1 + c2 * c2 + c3 * c3);
        r[0] = c0 / nc; r[1] = c1 / nc; r[2] = c2 / nc; r[3] = c3 / nc;
    }
}

/* 3x3 matrix of the SU(2) element r acting on rows/columns (i, j) */
static mat3 su2_embed(const double r[4], int i, int j)
{
    mat3 R = mat_identity();
    R.m[i][i] = r[0] + I * r[3];
    R.m[i][j] = r[2] + I * r[1];
    R.m[j][i] = -r[2] + I * r[1];
    R.m[j][j] = r[0] - I * r[3];
    return R;
}

/* The local update of one site (Sec. 3 with Eqs. (7)-(9)).
 * links: 8 links of 18 doubles, U_0(x)..U_3(x) then U_0(x-0)..U_3(x-3); they
 * are replaced by G U_mu(x) and U_mu(x-mu) G^dag.  sr[k] != 0 makes subgroup k
 * take the stochastic-relaxation square.  G (18 doubles) is returned when
 * G_out is not NULL. */
static void local_update_from(double *links, double omega, const int sr[3], double *G_out,
                              int mu_first)
{
    static const int sub[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    mat3 K = mat_zero();
    for (int mu = mu_first; mu < 4; ++mu) {
        mat3 uf = mat_load(links + 18 * mu);
        mat3 ub = mat_load(links + 18 * (4 + mu));
        mat3 ubd = mat_dag(&ub);
        K = mat_add(&K, &uf);
        K = mat_add(&K, &ubd);
    }
    mat3 W = K, G = mat_identity();
    for (int k = 0; k < 3; ++k) {
        int i = sub[k][0], j = sub[k][1];
        double w[8] = {creal(W.m[i][i]), cimag(W.m[i][i]), creal(W.m[i][j]), cimag(W.m[i][j]),
                       creal(W.m[j][i]), cimag(W.m[j][i]), creal(W.m[j][j]), cimag(W.m[j][j])};
        double r[4];
        orc_su2_step(w, omega, sr ? sr[k] : 0, r);
        mat3 R = su2_embed(r, i, j);
        W = mat_mul(&R, &W);
        G = mat_mul(&R, &G);
    }
    mat3 Gd = mat_dag(&G);
    for (int mu = 0; mu < 4; ++mu) {
        mat3 uf = mat_load(links + 18 * mu);
        mat3 ub = mat_load(links + 18 * (4 + mu));
        mat3 nf = mat_mul(&G, &uf);
        mat3 nb = mat_mul(&ub, &Gd);
        mat_store(&nf, links + 18 * mu);
        mat_store(&nb, links + 18 * (4 + mu));
    }
    if (G_out) mat_store(&G, G_out);
}

void orc_local_update(double *links, double omega, const int sr[3], double *G_out)
{
    local_update_from(links, omega, sr, G_out, 0);
}

/* Coulomb gauge: the same local update with K(x) from the 6 spatial links only
 * (the functional holds the spatial links of each timeslice), and G still
 * applied to all 8 links, the temporal ones included (a gauge transformation
 * acts on every link). */
void orc_local_update_coulomb(double *links, double omega, const int sr[3], double *G_out)
{
    local_update_from(links, omega, sr, G_out, 1);
}

/* Stochastic-relaxation coin flips of one site update: Philox keyed by the
 * seed with counter (site, sweep, instance, 3); subgroup k squares when word k
 * is below floor(p 2^32) (both compared as 64-bit integers, so p = 1 always
 * squares and p = 0 never does). */
void orc_sr_decisions(uint64_t seed, int64_t s, uint64_t sweep, uint32_t instance,
                      double p, int sr[3])
{
    uint32_t w[4];
    philox_seeded(seed, (uint32_t)s, (uint32_t)sweep, instance, 3u, w);
    uint64_t thr = (uint64_t)floor(p * 4294967296.0);
    for (int k = 0; k < 3; ++k) sr[k] = ((uint64_t)w[k] < thr) ? 1 : 0;
}

static void update_site_from(const lattice *lat, double *U, int64_t s, double omega, double p,
                             uint64_t seed, uint64_t sweep, uint32_t instance, int mu_first)
{
    double links[8 * 18];
    int64_t back[4];
    for (int mu = 0; mu < 4; ++mu) {
        back[mu] = site_neighbor(lat, s, mu, -1);
        memcpy(links + 18 * mu, link_cptr(U, s, mu), 18 * sizeof(double));
        memcpy(links + 18 * (4 + mu), link_cptr(U, back[mu], mu), 18 * sizeof(double));
    }
    int sr[3] = {0, 0, 0};
    if (p > 0.0) orc_sr_decisions(seed, s, sweep, instance, p, sr);
    local_update_from(links, omega, sr, NULL, mu_first);
    for (int mu = 0; mu < 4; ++mu) {
        memcpy(link_ptr(U, s, mu), links + 18 * mu, 18 * sizeof(double));
        memcpy(link_ptr(U, back[mu], mu), links + 18 * (4 + mu), 18 * sizeof(double));
    }
}

static void update_site(const lattice *lat, double *U, int64_t s, double omega, double p,
                        uint64_t seed, uint64_t sweep, uint32_t instance)
{
    update_site_from(lat, U, s, omega, p, seed, sweep, instance, 0);
}

/* One half-sweep: every site of the given parity gets its local update.  The
 * sites of one parity share no link, so the order is immaterial (Sec. 3); with
 * order == NULL the sites are visited in index order (in parallel), otherwise
 * in the n_order sites listed (serially).  Returns -1 when a listed site has
 * the other parity, else 0. */
int orc_half_sweep(const int dims[4], double *U, int parity, double omega, double p,
                   uint64_t seed, uint64_t sweep, uint32_t instance,
                   const int64_t *order, int64_t n_order)
{
    lattice lat = make_lattice(dims);
    if (order) {
        for (int64_t k = 0; k < n_order; ++k)
            if (site_parity(&lat, order[k]) != parity) return -1;
        for (int64_t k = 0; k < n_order; ++k)
            update_site(&lat, U, order[k], omega, p, seed, sweep, instance);
        return 0;
    }
    #pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < lat.V; ++s)
        if (site_parity(&lat, s) == parity)
            update_site(&lat, U, s, omega, p, seed, sweep, instance);
    return 0;
}

/* A full sweep: parity 0, then parity 1 (Sec. 4: the parities in turn). */
void orc_sweep(const int dims[4], double *U, double omega, double p, uint64_t seed,
               uint64_t sweep, uint32_t instance)
{
    orc_half_sweep(dims, U, 0, omega, p, seed, sweep, instance, NULL, 0);
    orc_half_sweep(dims, U, 1, omega, p, seed, sweep, instance, NULL, 0);
}

/* Coulomb-gauge half-sweep: every site of the 4-D parity whose timeslice is
 * active (slice_active == NULL: all) gets the Coulomb local update.  Sites of
 * one 4-D parity share no link, temporal links included, so the timeslices are
 * relaxed together while their functionals stay independent. */
void orc_half_sweep_coulomb(const int dims[4], double *U, int parity, double omega, double p,
                            uint64_t seed, uint64_t sweep, uint32_t instance,
                            const unsigned char *slice_active)
{
    lattice lat = make_lattice(dims);
    const int64_t V3 = lat.V / lat.L[0];
    #pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < lat.V; ++s)
        if (site_parity(&lat, s) == parity && (!slice_active || slice_active[s / V3]))
            update_site_from(&lat, U, s, omega, p, seed, sweep, instance, 1);
}

void orc_reunitarize(int64_t n_links, double *U)
{
    #pragma omp parallel for schedule(static)
    for (int64_t l = 0; l < n_links; ++l) {
        mat3 a = mat_load(U + 18 * l);
        mat3 r = mat_reunitarize(&a);
        mat_store(&r, U + 18 * l);
    }
}

/* ------------------------------------------------------------------------ */
/* Measurements                                                              */
/* ------------------------------------------------------------------------ */

/* A_mu(x) = (U - U^dag)/(2i) minus a third of its trace */
static mat3 gauge_potential(const mat3 *u)
{
    mat3 ud = mat_dag(u);
    mat3 d = mat_sub(u, &ud);
    mat3 A = mat_scale(&d, 1.0 / (2.0 * I));
    cplx tr = mat_trace(&A) / 3.0;
    for (int i = 0; i < 3; ++i) A.m[i][i] -= tr;
    return A;
}

/* F of Eq. (2) at g = 1 (N_c = 3, N_d = 4) and theta of Eqs. (4)-(5). */
void orc_measure(const int dims[4], const double *U, double *F, double *theta)
{
    lattice lat = make_lattice(dims);
    double *f_site = (double *)malloc(sizeof(double) * lat.V);
    double *t_site = (double *)malloc(sizeof(double) * lat.V);
    #pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < lat.V; ++s) {
        double fs = 0.0;
        mat3 Delta = mat_zero();
        for (int mu = 0; mu < 4; ++mu) {
            mat3 uf = mat_load(link_cptr(U, s, mu));
            mat3 ub = mat_load(link_cptr(U, site_neighbor(&lat, s, mu, -1), mu));
            fs += creal(mat_trace(&uf));
            mat3 Af = gauge_potential(&uf), Ab = gauge_potential(&ub);
            mat3 d = mat_sub(&Af, &Ab);
            Delta = mat_add(&Delta, &d);
        }
        mat3 Dd = mat_dag(&Delta);
        mat3 DDd = mat_mul(&Delta, &Dd);
        f_site[s] = fs;
        t_site[s] = creal(mat_trace(&DDd));
    }
    double fsum = 0.0, tsum = 0.0;
    for (int64_t s = 0; s < lat.V; ++s) { fsum += f_site[s]; tsum += t_site[s]; }
    free(f_site);
    free(t_site);
    *F = fsum / (3.0 * 4.0 * (double)lat.V);
    *theta = tsum / (3.0 * (double)lat.V);
}

/* Coulomb gauge, per timeslice t (spatial directions i = 1, 2, 3 only):
 * F_C(t) = (1/(3*3*V3)) sum_{x in t, i} Re tr U_i(x) and
 * theta_C(t) = (1/(3*V3)) sum_{x in t} tr[Delta_C Delta_C^dag] with
 * Delta_C(x) = sum_i A_i(x) - A_i(x - i).  F and theta hold Lt values each. */
void orc_measure_coulomb(const int dims[4], const double *U, double *F, double *theta)
{
    lattice lat = make_lattice(dims);
    const int64_t V3 = lat.V / lat.L[0];
    double *f_site = (double *)malloc(sizeof(double) * lat.V);
    double *t_site = (double *)malloc(sizeof(double) * lat.V);
    #pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < lat.V; ++s) {
        double fs = 0.0;
        mat3 Delta = mat_zero();
        for (int mu = 1; mu < 4; ++mu) {
            mat3 uf = mat_load(link_cptr(U, s, mu));
            mat3 ub = mat_load(link_cptr(U, site_neighbor(&lat, s, mu, -1), mu));
            fs += creal(mat_trace(&uf));
            mat3 Af = gauge_potential(&uf), Ab = gauge_potential(&ub);
            mat3 d = mat_sub(&Af, &Ab);
            Delta = mat_add(&Delta, &d);
        }
        mat3 Dd = mat_dag(&Delta);
        mat3 DDd = mat_mul(&Delta, &Dd);
        f_site[s] = fs;
        t_site[s] = creal(mat_trace(&DDd));
    }
    for (int t = 0; t < lat.L[0]; ++t) {
        double fsum = 0.0, tsum = 0.0;
        for (int64_t s = t * V3; s < (t + 1) * V3; ++s) { fsum += f_site[s]; tsum += t_site[s]; }
        F[t] = fsum / (3.0 * 3.0 * (double)V3);
        theta[t] = tsum / (3.0 * (double)V3);
    }
    free(f_site);
    free(t_site);
}

/* Average of (1/3) Re tr of the R x T rectangular loop in the (mu, nu) plane:
 * R steps along mu, T along nu, R back along mu, T back along nu. */
double orc_wilson_loop(const int dims[4], const double *U, int mu, int nu, int R, int T)
{
    lattice lat = make_lattice(dims);
    double *w_site = (double *)malloc(sizeof(double) * lat.V);
    #pragma omp parallel for schedule(static)
    for (int64_t s = 0; s < lat.V; ++s) {
        mat3 P = mat_identity();
        int64_t y = s;
        for (int k = 0; k < R; ++k) {
            mat3 u = mat_load(link_cptr(U, y, mu));
            P = mat_mul(&P, &u);
            y = site_neighbor(&lat, y, mu, +1);
        }
        for (int k = 0; k < T; ++k) {
            mat3 u = mat_load(link_cptr(U, y, nu));
            P = mat_mul(&P, &u);
            y = site_neighbor(&lat, y, nu, +1);
        }
        for (int k = 0; k < R; ++k) {
            y = site_neighbor(&lat, y, mu, -1);
            mat3 u = mat_load(link_cptr(U, y, mu));
            mat3 ud = mat_dag(&u);
            P = mat_mul(&P, &ud);
        }
        for (int k = 0; k < T; ++k) {
            y = site_neighbor(&lat, y, nu, -1);
            mat3 u = mat_load(link_cptr(U, y, nu));
            mat3 ud = mat_dag(&u);
            P = mat_mul(&P, &ud);
        }
        w_site[s] = creal(mat_trace(&P)) / 3.0;
    }
    double sum = 0.0;
    for (int64_t s = 0; s < lat.V; ++s) sum += w_site[s];
    free(w_site);
    return sum / (double)lat.V;
}

/* Plaquette: the 1x1 loop averaged over the six planes. */
double orc_plaquette(const int dims[4], const double *U)
{
    double sum = 0.0;
    for (int mu = 0; mu < 4; ++mu)
        for (int nu = mu + 1; nu < 4; ++nu)
            sum += orc_wilson_loop(dims, U, mu, nu, 1, 1);
    return sum / 6.0;
}

/* ------------------------------------------------------------------------ */
/* Simulated annealing.  The paper lists it among the supported methods        */
/* (Sec. 1) without its details, which it leaves to a reference not included. */
/* Reading used here: the SU(2) step of each Cabibbo-Marinari subgroup draws   */
/* r from the Boltzmann weight exp(Re tr[s(r) w] / T) on SU(2) (a heat bath at */
/* temperature T for the local functional of Eq. (7)); T falls linearly over   */
/* the annealing sweeps, and overrelaxation then takes the result to the gauge */
/* precision (Sec. 4).                                                         */
/* ------------------------------------------------------------------------ */

#define SA_TRIALS 64      /* accept-reject attempts per subgroup step */
#define SA_SWITCH 0.7     /* alpha below which the uniform proposal is used */

/* A uniform variate in (0,1) from one Philox word: (w + 1/2) 2^-32. */
static double unit_uniform(uint32_t w) { return ((double)w + 0.5) / 4294967296.0; }

/* Philox tag (fourth counter word) of trial t of subgroup k, and of the
 * subgroup's direction draw (t = 0xFFFF). */
static uint32_t sa_tag(int k, uint32_t t) { return ((uint32_t)(k + 1) << 16) | t; }

/* x0 in [-1, 1] with density proportional to sqrt(1 - x0^2) exp(alpha x0):
 * the component along the maximum of an SU(2) element drawn from
 * exp(alpha <x, 1>) times the Haar measure (the Haar measure of SU(2) = S^3
 * gives x0 the density sqrt(1 - x0^2)).  Each trial uses the words of one
 * Philox call keyed by the seed with counter (site, sweep, instance,
 * sa_tag(k, trial)).
 *  - alpha >= SA_SWITCH, Kennedy-Pendleton (Phys. Lett. B 156 (1985) 393):
 *    x0 = 1 - 2 l with l = -(ln u1 + cos^2(2 pi u2) ln u3) / (2 alpha), a
 *    Gamma(3/2) variate of rate 2 alpha, accepted when u4^2 <= 1 - l.
 *  - alpha < SA_SWITCH: x0 = 2 u1 - 1 accepted when
 *    u2^2 <= (1 - x0^2) exp(2 alpha (x0 - 1)).
 * Both accept at least 40 % of trials for every alpha.  Returns the trials
 * used; when all SA_TRIALS fail (probability below 1e-14) x0 = 1 and the
 * count is SA_TRIALS + 1. */
static int heatbath_x0(double alpha, uint64_t seed, uint32_t s, uint32_t sweep, uint32_t instance, int k,
                       double *x0)
{
    for (uint32_t t = 0; t < SA_TRIALS; ++t) {
        uint32_t w[4];
        philox_seeded(seed, s, sweep, instance, sa_tag(k, t), w);
        const double u1 = unit_uniform(w[0]), u2 = unit_uniform(w[1]);
        const double u3 = unit_uniform(w[2]), u4 = unit_uniform(w[3]);
        if (alpha >= SA_SWITCH) {
            const double c = cos(2.0 * M_PI * u2);
            const double l = -(log(u1) + c * c * log(u3)) / (2.0 * alpha);
            if (u4 * u4 <= 1.0 - l) {
                *x0 = 1.0 - 2.0 * l;
                return (int)t + 1;
            }
        } else {
            const double x = 2.0 * u1 - 1.0;
            if (u2 * u2 <= (1.0 - x * x) * exp(2.0 * alpha * (x - 1.0))) {
                *x0 = x;
                return (int)t + 1;
            }
        }
    }
    *x0 = 1.0;
    return SA_TRIALS + 1;
}

/* The heat-bath step of one subgroup.  w as in orc_su2_step; with a its
 * quaternion projection, Re tr[s(r) w] = 2 |a| <r, b>, b = (a0, -a)/|a| the
 * maximum of Eq. (9) (b = 1 when a = 0).  Writing r = x b (quaternion
 * product, s(r) = s(x) s(b)), <r, b> = x0 and the Haar measure is unchanged,
 * so x is drawn from exp(alpha x0) dHaar(x) with alpha = 2 |a| / T: x0 by
 * heatbath_x0, the direction of (x1, x2, x3) uniform on the sphere of radius
 * sqrt(1 - x0^2) (cos theta = 2 v1 - 1, phi = 2 pi v2 from the words of the
 * call with tag sa_tag(k, 0xFFFF)).  Returns the accept-reject trials used;
 * r = (r0, r1, r2, r3). */
int orc_su2_heatbath(const double w[8], double T, uint64_t seed, int64_t s, uint64_t sweep,
                     uint32_t instance, int k, double r[4])
{
    double a0 = 0.5 * (w[0] + w[6]);
    double a3 = 0.5 * (w[1] - w[7]);
    double a1 = 0.5 * (w[3] + w[5]);
    double a2 = 0.5 * (w[2] - w[4]);
    double na = sqrt(a0 * a0 + a1 * a1 + a2 * a2 + a3 * a3);
    double b0 = 1.0, b1 = 0.0, b2 = 0.0, b3 = 0.0;
    if (na > 0.0) { b0 = a0 / na; b1 = -a1 / na; b2 = -a2 / na; b3 = -a3 / na; }
    const double alpha = 2.0 * na / T;
    double x0;
    const int trials = heatbath_x0(alpha, seed, (uint32_t)s, (uint32_t)sweep, instance, k, &x0);
    uint32_t v[4];
    philox_seeded(seed, (uint32_t)s, (uint32_t)sweep, instance, sa_tag(k, 0xFFFFu), v);
    const double ct = 2.0 * unit_uniform(v[0]) - 1.0;
    const double phi = 2.0 * M_PI * unit_uniform(v[1]);
    const double st = sqrt(1.0 - ct * ct);
    const double rad = sqrt(fmax(0.0, 1.0 - x0 * x0));
    const double x1 = rad * st * cos(phi), x2 = rad * st * sin(phi), x3 = rad * ct;
    /* s(x) s(b) = (x0 b0 - x.b) + i (x0 b + b0 x - x cross b).sigma */
    r[0] = x0 * b0 - (x1 * b1 + x2 * b2 + x3 * b3);
    r[1] = x0 * b1 + b0 * x1 - (x2 * b3 - x3 * b2);
    r[2] = x0 * b2 + b0 * x2 - (x3 * b1 - x1 * b3);
    r[3] = x0 * b3 + b0 * x3 - (x1 * b2 - x2 * b1);
    return trials;
}

/* The annealing update of one site: K(x) as in the local update (Eq. (8)),
 * the three subgroups in order with the heat-bath step, G applied to the 8
 * links.  Returns the accept-reject trials of the three steps. */
static int64_t local_update_sa(double *links, double T, uint64_t seed, int64_t s, uint64_t sweep,
                               uint32_t instance)
{
    static const int sub[3][2] = {{0, 1}, {0, 2}, {1, 2}};
    mat3 K = mat_zero();
    for (int mu = 0; mu < 4; ++mu) {
        mat3 uf = mat_load(links + 18 * mu);
        mat3 ub = mat_load(links + 18 * (4 + mu));
        mat3 ubd = mat_dag(&ub);
        K = mat_add(&K, &uf);
        K = mat_add(&K, &ubd);
    }
    mat3 W = K, G = mat_identity();
    int64_t trials = 0;
    for (int k = 0; k < 3; ++k) {
        int i = sub[k][0], j = sub[k][1];
        double w[8] = {creal(W.m[i][i]), cimag(W.m[i][i]), creal(W.m[i][j]), cimag(W.m[i][j]),
                       creal(W.m[j][i]), cimag(W.m[j][i]), creal(W.m[j][j]), cimag(W.m[j][j])};
        double r[4];
        trials += orc_su2_heatbath(w, T, seed, s, sweep, instance, k, r);
        mat3 R = su2_embed(r, i, j);
        W = mat_mul(&R, &W);
        G = mat_mul(&R, &G);
    }
    mat3 Gd = mat_dag(&G);
    for (int mu = 0; mu < 4; ++mu) {
        mat3 uf = mat_load(links + 18 * mu);
        mat3 ub = mat_load(links + 18 * (4 + mu));
        mat3 nf = mat_mul(&G, &uf);
        mat3 nb = mat_mul(&ub, &Gd);
        mat_store(&nf, links + 18 * mu);
        mat_store(&nb, links + 18 * (4 + mu));
    }
    return trials;
}

/* The annealing update of the 8 links of site s (forward, then backward, as
 * in orc_local_update) with the Philox counters of site s; returns the
 * trials. */
int64_t orc_local_update_sa(double *links, double T, uint64_t seed, int64_t s, uint64_t sweep,
                            uint32_t instance)
{
    return local_update_sa(links, T, seed, s, sweep, instance);
}

/* One annealing half-sweep at temperature T: every site of the parity gets
 * its heat-bath update (same-parity sites share no link, Sec. 3).  Returns the
 * total accept-reject trials. */
int64_t orc_half_sweep_sa(const int dims[4], double *U, int parity, double T, uint64_t seed,
                          uint64_t sweep, uint32_t instance)
{
    lattice lat = make_lattice(dims);
    int64_t trials = 0;
    #pragma omp parallel for schedule(static) reduction(+:trials)
    for (int64_t s = 0; s < lat.V; ++s) {
        if (site_parity(&lat, s) != parity) continue;
        double links[8 * 18];
        int64_t back[4];
        for (int mu = 0; mu < 4; ++mu) {
            back[mu] = site_neighbor(&lat, s, mu, -1);
            memcpy(links + 18 * mu, link_cptr(U, s, mu), 18 * sizeof(double));
            memcpy(links + 18 * (4 + mu), link_cptr(U, back[mu], mu), 18 * sizeof(double));
        }
        trials += local_update_sa(links, T, seed, s, sweep, instance);
        for (int mu = 0; mu < 4; ++mu) {
            memcpy(link_ptr(U, s, mu), links + 18 * mu, 18 * sizeof(double));
            memcpy(link_ptr(U, back[mu], mu), links + 18 * (4 + mu), 18 * sizeof(double));
        }
    }
    return trials;
}

/* Temperature of annealing sweep n of n_sweeps: linear from T_start (n = 0)
 * to T_end (n = n_sweeps - 1). */
double orc_anneal_temperature(int64_t n, int64_t n_sweeps, double T_start, double T_end)
{
    if (n_sweeps <= 1) return T_start;
    const double f = (double)n / (double)(n_sweeps - 1);
    return T_start * (1.0 - f) + T_end * f;
}

/* n_sweeps annealing sweeps (parity 0, then 1) with the linear schedule; sweep
 * n uses Philox counter sweep0 + n; the links are reunitarized after every
 * 20 sweeps and at the end.  Returns the total accept-reject trials. */
int64_t orc_anneal(const int dims[4], double *U, int64_t n_sweeps, double T_start, double T_end,
                   uint64_t seed, uint64_t sweep0, uint32_t instance)
{
    lattice lat = make_lattice(dims);
    int64_t trials = 0;
    for (int64_t n = 0; n < n_sweeps; ++n) {
        const double T = orc_anneal_temperature(n, n_sweeps, T_start, T_end);
        trials += orc_half_sweep_sa(dims, U, 0, T, seed, sweep0 + (uint64_t)n, instance);
        trials += orc_half_sweep_sa(dims, U, 1, T, seed, sweep0 + (uint64_t)n, instance);
        if ((n + 1) % 20 == 0 || n + 1 == n_sweeps) orc_reunitarize(lat.V * 4, U);
    }
    return trials;
}

/* ------------------------------------------------------------------------ */
/* Iterate until the requested precision (Sec. 4)                             */
/* ------------------------------------------------------------------------ */

/* Full sweeps (parity 0 then 1) with sweep counter running from 0; every
 * check_every sweeps the links are reunitarized (when reunitarize != 0) and
 * F, theta measured; the run stops at the first measurement with theta <
 * theta_target, or after max_sweeps.  Measurement 0 is taken on the input.
 * history (may be NULL) receives (sweeps, F, theta) triples, up to
 * history_cap of them.  Returns 0 when converged, 1 when max_sweeps was hit. */
int orc_gauge_fix(const int dims[4], double *U, double omega, double p, double theta_target,
                  int check_every, int reunitarize, int64_t max_sweeps, uint64_t seed,
                  uint32_t instance, int64_t *sweeps_out, double *F_out, double *theta_out,
                  double *history, int64_t history_cap, int64_t *n_history)
{
    lattice lat = make_lattice(dims);
    int64_t sweeps = 0, nh = 0;
    double F, theta;
    orc_measure(dims, U, &F, &theta);
    if (history && nh < history_cap) {
        history[3 * nh] = 0.0; history[3 * nh + 1] = F; history[3 * nh + 2] = theta; ++nh;
    }
    int status = 1;
    if (theta < theta_target) status = 0;
    while (status != 0 && sweeps < max_sweeps) {
        for (int k = 0; k < check_every && sweeps < max_sweeps; ++k) {
            orc_sweep(dims, U, omega, p, seed, (uint64_t)sweeps, instance);
            ++sweeps;
        }
        if (reunitarize) orc_reunitarize(lat.V * 4, U);
        orc_measure(dims, U, &F, &theta);
        if (history && nh < history_cap) {
            history[3 * nh] = (double)sweeps; history[3 * nh + 1] = F; history[3 * nh + 2] = theta;
            ++nh;
        }
        if (theta < theta_target) status = 0;
    }
    *sweeps_out = sweeps;
    *F_out = F;
    *theta_out = theta;
    if (n_history) *n_history = nh;
    return status;
}

/* Coulomb gauge fixing of every timeslice: full sweeps (parity 0 then 1) of
 * the timeslices still active; every check_every sweeps reunitarize (all
 * links) and measure theta_C(t); a timeslice stops (is frozen) at its first
 * measurement with theta_C(t) < theta_target.  Outputs per timeslice: the
 * sweeps it took (sweeps_t, as doubles), F_C(t), theta_C(t).  Returns 0 when
 * every timeslice converged, 1 when max_sweeps was hit first. */
int orc_coulomb_gauge_fix(const int dims[4], double *U, double omega, double p, double theta_target,
                          int check_every, int reunitarize, int64_t max_sweeps, uint64_t seed,
                          uint32_t instance, double *sweeps_t, double *F_t, double *theta_t,
                          int64_t *sweeps_out)
{
    lattice lat = make_lattice(dims);
    const int Lt = lat.L[0];
    unsigned char *active = (unsigned char *)malloc((size_t)Lt);
    orc_measure_coulomb(dims, U, F_t, theta_t);
    int n_active = 0;
    for (int t = 0; t < Lt; ++t) {
        active[t] = theta_t[t] < theta_target ? 0 : 1;
        sweeps_t[t] = 0.0;
        n_active += active[t];
    }
    int64_t sweeps = 0;
    while (n_active > 0 && sweeps < max_sweeps) {
        for (int k = 0; k < check_every && sweeps < max_sweeps; ++k) {
            orc_half_sweep_coulomb(dims, U, 0, omega, p, seed, (uint64_t)sweeps, instance, active);
            orc_half_sweep_coulomb(dims, U, 1, omega, p, seed, (uint64_t)sweeps, instance, active);
            ++sweeps;
        }
        if (reunitarize) orc_reunitarize(lat.V * 4, U);
        double *F = (double *)malloc(sizeof(double) * Lt);
        double *th = (double *)malloc(sizeof(double) * Lt);
        orc_measure_coulomb(dims, U, F, th);
        n_active = 0;
        for (int t = 0; t < Lt; ++t) {
            if (!active[t]) continue;
            F_t[t] = F[t];
            theta_t[t] = th[t];
            sweeps_t[t] = (double)sweeps;
            if (th[t] < theta_target) active[t] = 0;
            n_active += active[t];
        }
        free(F);
        free(th);
    }
    free(active);
    *sweeps_out = sweeps;
    return n_active > 0 ? 1 : 0;
}

/* Threads for the oracle's later parallel regions (n >= 1; a no-op without
   OpenMP).  Used only to time the oracle on one core beside all of them. */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* Number of OpenMP threads a parallel region of the oracle uses. */
int orc_num_threads(void)
{
    int n = 1;
    #pragma omp parallel
    {
        #pragma omp single
        {
#ifdef _OPENMP
            n = omp_get_num_threads();
#endif
        }
    }
    return n;
}
