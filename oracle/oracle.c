/*
 * oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, FP64 CPU reference of everything the domain-wall hot path
 * computes.  Only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library; the product path never does.  It shares no
 * code, header, table or constant with the HIP library.
 *
 * Everything is written from the definitions, on the full lexicographic
 * lattice, with explicit 4x4 gamma matrices and no spin projection:
 *
 *   site index   n = x + Lx*(y + Ly*(z + Lz*t)),  parity (x+y+z+t) mod 2
 *   fermion      psi[n][s][spin 4][colour 3]      (complex double)
 *   gauge        U[n][mu][row 3][col 3],           U_mu(x) links x -> x+mu
 *   half field   psi[cb][s][spin][colour], cb = n>>1 among sites of one parity
 *
 * Domain-wall operator (Moebius form; the paper never writes it out, it
 * follows Brower, Neff and Orginos):
 *   H psi(x)   = sum_mu (1-g_mu) U_mu(x) psi(x+mu) + (1+g_mu) U_mu(x-mu)^+ psi(x-mu)
 *   D_W        = (4 - M5) - H/2
 *   P5 psi_s   = P_- psi_{s+1} + P_+ psi_{s-1},  psi_Ls = -mf psi_0, psi_-1 = -mf psi_{Ls-1}
 *   D5         = (b D_W + 1) + (c D_W - 1) P5
 *   D5^+       = (b D_W^+ + 1) + P5^+ (c D_W^+ - 1)
 * Dirichlet block (Sec. 2.4, "Results"): links leaving the block through a
 * face are set to zero, U_mu(x) = 0 for x_mu = L_mu - 1.
 * Red-black Schur complement on odd sites (the "usual red-black
 * preconditioned" solve of Sec. 2.3):
 *   Mpc = Moo - Moe Mee^-1 Meo, every block read off D5 by restriction.
 *
 * Parity of each function is pinned in tests/ against closed forms and
 * invariants (free field, Wilson limit, overlap determinant, gamma5 R5
 * hermiticity, gauge covariance, Schur determinant, eq. (ddrhmc)).
 */
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* ---------------------------------------------------------------- gammas */

static cplx G[4][4][4];   /* G[mu][alpha][beta], chiral basis */
static cplx G5[4][4];
static cplx PP[4][4];     /* (1 + g5)/2 */
static cplx PM[4][4];     /* (1 - g5)/2 */
static int g_ready = 0;

static void mat4_mul(cplx a[4][4], cplx b[4][4], cplx out[4][4])
{
    cplx t[4][4];
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            cplx s = 0;
            for (int k = 0; k < 4; k++) s += a[i][k] * b[k][j];
            t[i][j] = s;
        }
    memcpy(out, t, sizeof(t));
}

/* gamma_k = [[0, -i sigma_k], [i sigma_k, 0]] (k = x,y,z), gamma_t = [[0,1],[1,0]] */
static void init_gamma(void)
{
    if (g_ready) return;
    cplx sig[3][2][2] = {
        {{0, 1}, {1, 0}},
        {{0, -I}, {I, 0}},
        {{1, 0}, {0, -1}},
    };
    memset(G, 0, sizeof(G));
    for (int k = 0; k < 3; k++)
        for (int a = 0; a < 2; a++)
            for (int b = 0; b < 2; b++) {
                G[k][a][b + 2] = -I * sig[k][a][b];
                G[k][a + 2][b] = I * sig[k][a][b];
            }
    for (int a = 0; a < 2; a++) {
        G[3][a][a + 2] = 1;
        G[3][a + 2][a] = 1;
    }
    mat4_mul(G[0], G[1], G5);
    mat4_mul(G5, G[2], G5);
    mat4_mul(G5, G[3], G5);
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) {
            cplx id = (i == j) ? 1.0 : 0.0;
            PP[i][j] = 0.5 * (id + G5[i][j]);
            PM[i][j] = 0.5 * (id - G5[i][j]);
        }
    g_ready = 1;
}

/* exported so tests can check the Clifford algebra of the table itself */
/* threads the parallel loops of this library run on */
int or_num_threads(void) { return omp_get_max_threads(); }

/* Threads of the following parallel loops (the CPU baseline times one and all). */
void or_set_num_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }

void or_gamma(int mu, double *out /* 4x4 complex */)
{
    init_gamma();
    cplx *o = (cplx *)out;
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++) o[i * 4 + j] = (mu < 4) ? G[mu][i][j] : G5[i][j];
}

/* ------------------------------------------------------------ geometry */

static long vol(const int *L) { return (long)L[0] * L[1] * L[2] * L[3]; }

static void coords(const int *L, long n, int x[4])
{
    for (int mu = 0; mu < 4; mu++) {
        x[mu] = (int)(n % L[mu]);
        n /= L[mu];
    }
}

static long index4(const int *L, const int x[4])
{
    return x[0] + (long)L[0] * (x[1] + (long)L[1] * (x[2] + (long)L[2] * x[3]));
}

static long shifted(const int *L, long n, int mu, int step)
{
    int x[4];
    coords(L, n, x);
    x[mu] = (x[mu] + step + L[mu]) % L[mu];
    return index4(L, x);
}

static int parity(const int *L, long n)
{
    int x[4];
    coords(L, n, x);
    return (x[0] + x[1] + x[2] + x[3]) & 1;
}

#define FIDX(n, s, sp, c, Ls) ((((long)(n) * (Ls) + (s)) * 4 + (sp)) * 3 + (c))
#define UIDX(n, mu, r, c) ((((long)(n) * 4 + (mu)) * 3 + (r)) * 3 + (c))

/* ------------------------------------------------------------ gauge */

/* Dirichlet block: zero U_mu(x) on the last slice x_mu = L_mu - 1 for each flagged mu. */
void or_dirichlet(const int *L, const int *mask, const double *Uin, double *Uout)
{
    const cplx *U = (const cplx *)Uin;
    cplx *O = (cplx *)Uout;
    long V = vol(L);
    for (long n = 0; n < V; n++) {
        int x[4];
        coords(L, n, x);
        for (int mu = 0; mu < 4; mu++)
            for (int k = 0; k < 9; k++) {
                long i = UIDX(n, mu, 0, 0) + k;
                O[i] = (mask[mu] && x[mu] == L[mu] - 1) ? 0.0 : U[i];
            }
    }
}

/* --------------------------------------------------------------- hop */

/* out = H in (dagger = 0) or H^+ in = g5 H g5 in (dagger = 1), every s slice. */
void or_hop(const int *L, int Ls, const double *Uin, const double *in_, double *out_, int dagger)
{
    init_gamma();
    const cplx *U = (const cplx *)Uin;
    const cplx *in = (const cplx *)in_;
    cplx *out = (cplx *)out_;
    long V = vol(L);
    double sf = dagger ? +1.0 : -1.0; /* forward projector 1 + sf*g_mu */
#pragma omp parallel for schedule(static)
    for (long n = 0; n < V; n++) {
        for (int s = 0; s < Ls; s++) {
            cplx acc[4][3];
            memset(acc, 0, sizeof(acc));
            for (int mu = 0; mu < 4; mu++) {
                long nf = shifted(L, n, mu, +1);
                long nb = shifted(L, n, mu, -1);
                cplx v[4][3], w[4][3];
                for (int sp = 0; sp < 4; sp++)
                    for (int a = 0; a < 3; a++) {
                        cplx sv = 0, sw = 0;
                        for (int b = 0; b < 3; b++) {
                            sv += U[UIDX(n, mu, a, b)] * in[FIDX(nf, s, sp, b, Ls)];
                            sw += conj(U[UIDX(nb, mu, b, a)]) * in[FIDX(nb, s, sp, b, Ls)];
                        }
                        v[sp][a] = sv;
                        w[sp][a] = sw;
                    }
                for (int al = 0; al < 4; al++)
                    for (int a = 0; a < 3; a++) {
                        cplx t = 0;
                        for (int be = 0; be < 4; be++) {
                            cplx id = (al == be) ? 1.0 : 0.0;
                            t += (id + sf * G[mu][al][be]) * v[be][a];
                            t += (id - sf * G[mu][al][be]) * w[be][a];
                        }
                        acc[al][a] += t;
                    }
            }
            for (int sp = 0; sp < 4; sp++)
                for (int a = 0; a < 3; a++) out[FIDX(n, s, sp, a, Ls)] = acc[sp][a];
        }
    }
}

/* D_W = (4 - M5) - H/2 (dagger: H -> H^+) on every s slice. */
void or_dw(const int *L, int Ls, double M5, const double *U, const double *in_, double *out_, int dagger)
{
    long N = vol(L) * Ls * 12;
    or_hop(L, Ls, U, in_, out_, dagger);
    const cplx *in = (const cplx *)in_;
    cplx *out = (cplx *)out_;
#pragma omp parallel for schedule(static)
    for (long i = 0; i < N; i++) out[i] = (4.0 - M5) * in[i] - 0.5 * out[i];
}

/* P5 (dagger = 0) or P5^+ (dagger = 1) on nsite 4D sites. */
static void p5(long nsite, int Ls, double mf, const cplx *in, cplx *out, int dagger)
{
    init_gamma();
#pragma omp parallel for schedule(static)
    for (long n = 0; n < nsite; n++)
        for (int s = 0; s < Ls; s++) {
            int su = s + 1, sd = s - 1;
            double fu = 1.0, fd = 1.0;
            if (su == Ls) { su = 0; fu = -mf; }
            if (sd < 0) { sd = Ls - 1; fd = -mf; }
            /* non-dagger: P_- from s+1, P_+ from s-1; dagger swaps the projectors */
            cplx (*Pu)[4] = dagger ? PP : PM;
            cplx (*Pd)[4] = dagger ? PM : PP;
            for (int al = 0; al < 4; al++)
                for (int a = 0; a < 3; a++) {
                    cplx t = 0;
                    for (int be = 0; be < 4; be++)
                        t += fu * Pu[al][be] * in[FIDX(n, su, be, a, Ls)] + fd * Pd[al][be] * in[FIDX(n, sd, be, a, Ls)];
                    out[FIDX(n, s, al, a, Ls)] = t;
                }
        }
}

void or_p5(long nsite, int Ls, double mf, const double *in, double *out, int dagger)
{
    p5(nsite, Ls, mf, (const cplx *)in, (cplx *)out, dagger);
}

/* D5 = (b D_W + 1) + (c D_W - 1) P5 ;  D5^+ = (b D_W^+ + 1) + P5^+ (c D_W^+ - 1). */
void or_d5(const int *L, int Ls, double b, double c, double M5, double mf, const double *U,
           const double *in_, double *out_, int dagger)
{
    long N = vol(L) * Ls * 12;
    const cplx *in = (const cplx *)in_;
    cplx *out = (cplx *)out_;
    cplx *t1 = malloc(N * sizeof(cplx));
    cplx *t2 = malloc(N * sizeof(cplx));
    if (!dagger) {
        cplx *t3 = malloc(N * sizeof(cplx));
        or_dw(L, Ls, M5, U, in_, (double *)t1, 0);  /* D_W psi      */
        p5(vol(L), Ls, mf, in, t2, 0);                /* P5 psi       */
        or_dw(L, Ls, M5, U, (double *)t2, (double *)t3, 0); /* D_W P5 psi */
#pragma omp parallel for schedule(static)
        for (long i = 0; i < N; i++) out[i] = b * t1[i] + in[i] + c * t3[i] - t2[i];
        free(t3);
    } else {
        or_dw(L, Ls, M5, U, in_, (double *)t1, 1);  /* D_W^+ psi */
#pragma omp parallel for schedule(static)
        for (long i = 0; i < N; i++) t2[i] = c * t1[i] - in[i];
        cplx *t3 = malloc(N * sizeof(cplx));
        p5(vol(L), Ls, mf, t2, t3, 1);
#pragma omp parallel for schedule(static)
        for (long i = 0; i < N; i++) out[i] = b * t1[i] + in[i] + t3[i];
        free(t3);
    }
    free(t1);
    free(t2);
}

/* ------------------------------------------------------------ sampled sites */

/* The same operators evaluated only at a list of 4D sites (all s), for checks
 * at lattice sizes where the full operator is too expensive for the CPU.  Each
 * sample gathers its 9-site neighbourhood into a small periodic-free buffer and
 * applies the definitions above to it. */

/* (H in)(n) or (H^+ in)(n) for n in sites; out[k][s][spin][colour] */
void or_hop_sites(const int *L, int Ls, const double *Uin, const double *in_, const long *sites, long nsite,
                  double *out_, int dagger)
{
    init_gamma();
    const cplx *U = (const cplx *)Uin;
    const cplx *in = (const cplx *)in_;
    cplx *out = (cplx *)out_;
    double sf = dagger ? +1.0 : -1.0;
#pragma omp parallel for schedule(static)
    for (long k = 0; k < nsite; k++) {
        long n = sites[k];
        for (int s = 0; s < Ls; s++) {
            cplx acc[4][3];
            memset(acc, 0, sizeof(acc));
            for (int mu = 0; mu < 4; mu++) {
                long nf = shifted(L, n, mu, +1), nb = shifted(L, n, mu, -1);
                for (int al = 0; al < 4; al++)
                    for (int a = 0; a < 3; a++) {
                        cplx t = 0;
                        for (int be = 0; be < 4; be++) {
                            cplx id = (al == be) ? 1.0 : 0.0;
                            cplx v = 0, w = 0;
                            for (int b = 0; b < 3; b++) {
                                v += U[UIDX(n, mu, a, b)] * in[FIDX(nf, s, be, b, Ls)];
                                w += conj(U[UIDX(nb, mu, b, a)]) * in[FIDX(nb, s, be, b, Ls)];
                            }
                            t += (id + sf * G[mu][al][be]) * v + (id - sf * G[mu][al][be]) * w;
                        }
                        acc[al][a] += t;
                    }
            }
            for (int sp = 0; sp < 4; sp++)
                for (int a = 0; a < 3; a++) out[((k * Ls + s) * 4 + sp) * 3 + a] = acc[sp][a];
        }
    }
}

/* (D5 in)(n) for n in sites (non-dagger), from
 * D5 = (b D_W + 1) + (c D_W - 1) P5 with D_W = (4 - M5) - H/2 */
void or_d5_sites(const int *L, int Ls, double b, double c, double M5, double mf, const double *U, const double *in_,
                 const long *sites, long nsite, double *out_)
{
    const cplx *in = (const cplx *)in_;
    cplx *out = (cplx *)out_;
    long per = (long)Ls * 12;
    /* P5 in at the 9 sites of each neighbourhood, then the hops at the centre */
    cplx *hop_in = malloc(nsite * per * sizeof(cplx));
    cplx *hop_p5 = malloc(nsite * per * sizeof(cplx));
    or_hop_sites(L, Ls, U, in_, sites, nsite, (double *)hop_in, 0);
    long V = vol(L);
    /* P5 applied on the full field is s-local; evaluate it on the whole field once */
    cplx *p5in = malloc(V * per * sizeof(cplx));
    p5(V, Ls, mf, in, p5in, 0);
    or_hop_sites(L, Ls, U, (const double *)p5in, sites, nsite, (double *)hop_p5, 0);
    for (long k = 0; k < nsite; k++) {
        long n = sites[k];
        for (long e = 0; e < per; e++) {
            cplx x = in[n * per + e], px = p5in[n * per + e];
            cplx dw = (4.0 - M5) * x - 0.5 * hop_in[k * per + e];
            cplx dwp = (4.0 - M5) * px - 0.5 * hop_p5[k * per + e];
            out[k * per + e] = b * dw + x + c * dwp - px;
        }
    }
    free(hop_in);
    free(hop_p5);
    free(p5in);
}

/* ------------------------------------------------------------ parity */

static long site_of_cb(const int *L, long cb, int p)
{
    long n = 2 * cb;
    return (parity(L, n) == p) ? n : n + 1;
}

void or_pick(const int *L, int Ls, const double *full_, int p, double *half_)
{
    const cplx *full = (const cplx *)full_;
    cplx *half = (cplx *)half_;
    long Vh = vol(L) / 2, per = (long)Ls * 12;
    for (long cb = 0; cb < Vh; cb++) memcpy(half + cb * per, full + site_of_cb(L, cb, p) * per, per * sizeof(cplx));
}

void or_embed(const int *L, int Ls, const double *half_, int p, double *full_)
{
    const cplx *half = (const cplx *)half_;
    cplx *full = (cplx *)full_;
    long Vh = vol(L) / 2, per = (long)Ls * 12;
    memset(full, 0, vol(L) * per * sizeof(cplx));
    for (long cb = 0; cb < Vh; cb++) memcpy(full + site_of_cb(L, cb, p) * per, half + cb * per, per * sizeof(cplx));
}

/* Mooee = d + e P5 (dagger: d + e P5^+), d = b(4-M5)+1, e = c(4-M5)-1, on nsite sites */
void or_mooee(long nsite, int Ls, double b, double c, double M5, double mf, const double *in_, double *out_, int dagger)
{
    double d = b * (4.0 - M5) + 1.0, e = c * (4.0 - M5) - 1.0;
    long N = nsite * Ls * 12;
    const cplx *in = (const cplx *)in_;
    cplx *out = (cplx *)out_;
    cplx *t = malloc(N * sizeof(cplx));
    p5(nsite, Ls, mf, in, t, dagger);
    for (long i = 0; i < N; i++) out[i] = d * in[i] + e * t[i];
    free(t);
}

/* Gauss-Jordan inverse of an n x n complex matrix with partial pivoting. */
static int invert(int n, cplx *A, cplx *Ainv)
{
    cplx *M = malloc((size_t)n * 2 * n * sizeof(cplx));
    for (int i = 0; i < n; i++)
        for (int j = 0; j < 2 * n; j++) M[i * 2 * n + j] = (j < n) ? A[i * n + j] : ((j - n == i) ? 1.0 : 0.0);
    for (int col = 0; col < n; col++) {
        int piv = col;
        for (int r = col + 1; r < n; r++)
            if (cabs(M[r * 2 * n + col]) > cabs(M[piv * 2 * n + col])) piv = r;
        if (cabs(M[piv * 2 * n + col]) == 0.0) { free(M); return -1; }
        if (piv != col)
            for (int j = 0; j < 2 * n; j++) {
                cplx t = M[col * 2 * n + j];
                M[col * 2 * n + j] = M[piv * 2 * n + j];
                M[piv * 2 * n + j] = t;
            }
        cplx inv = 1.0 / M[col * 2 * n + col];
        for (int j = 0; j < 2 * n; j++) M[col * 2 * n + j] *= inv;
        for (int r = 0; r < n; r++) {
            if (r == col) continue;
            cplx f = M[r * 2 * n + col];
            if (f == 0.0) continue;
            for (int j = 0; j < 2 * n; j++) M[r * 2 * n + j] -= f * M[col * 2 * n + j];
        }
    }
    for (int i = 0; i < n; i++)
        for (int j = 0; j < n; j++) Ainv[i * n + j] = M[i * 2 * n + n + j];
    free(M);
    return 0;
}

/* Mooee^-1 (dagger: (Mooee^+)^-1): the one-site (12 Ls)^2 matrix of Mooee is
 * read off by applying it to unit vectors, inverted numerically, and applied
 * to every site.  No closed form is used here. */
void or_mooeeinv(long nsite, int Ls, double b, double c, double M5, double mf, const double *in_, double *out_, int dagger)
{
    int m = 12 * Ls;
    cplx *A = malloc((size_t)m * m * sizeof(cplx));
    cplx *Ai = malloc((size_t)m * m * sizeof(cplx));
    cplx *e = calloc(m, sizeof(cplx));
    cplx *col = malloc(m * sizeof(cplx));
    for (int j = 0; j < m; j++) {
        memset(e, 0, m * sizeof(cplx));
        e[j] = 1.0;
        or_mooee(1, Ls, b, c, M5, mf, (const double *)e, (double *)col, dagger);
        for (int i = 0; i < m; i++) A[i * m + j] = col[i];
    }
    invert(m, A, Ai);
    const cplx *in = (const cplx *)in_;
    cplx *out = (cplx *)out_;
#pragma omp parallel for schedule(static)
    for (long n = 0; n < nsite; n++)
        for (int i = 0; i < m; i++) {
            cplx t = 0;
            for (int j = 0; j < m; j++) t += Ai[i * m + j] * in[n * m + j];
            out[n * m + i] = t;
        }
    free(A); free(Ai); free(e); free(col);
}

/* M_{p_out, p_in} = restriction of D5 (or D5^+) from parity p_in to parity p_out:
 * embed the half field, apply the full operator, pick the other parity. */
void or_meo(const int *L, int Ls, double b, double c, double M5, double mf, const double *U,
            const double *in_half, int p_in, double *out_half, int dagger)
{
    long N = vol(L) * Ls * 12;
    double *f1 = malloc(N * sizeof(cplx));
    double *f2 = malloc(N * sizeof(cplx));
    or_embed(L, Ls, in_half, p_in, f1);
    or_d5(L, Ls, b, c, M5, mf, U, f1, f2, dagger);
    or_pick(L, Ls, f2, 1 - p_in, out_half);
    free(f1);
    free(f2);
}

/* Schur complement on odd sites:
 *   Mpc   = Moo - Moe Mee^-1 Meo
 *   Mpc^+ = Moo^+ - (Meo)^+ (Mee^-1)^+ (Moe)^+, every block read off D5^+. */
void or_mpc(const int *L, int Ls, double b, double c, double M5, double mf, const double *U,
            const double *in_odd, double *out_odd, int dagger)
{
    long Nh = vol(L) / 2 * Ls * 12;
    cplx *te = malloc(Nh * sizeof(cplx));
    cplx *te2 = malloc(Nh * sizeof(cplx));
    cplx *to = malloc(Nh * sizeof(cplx));
    or_meo(L, Ls, b, c, M5, mf, U, in_odd, 1, (double *)te, dagger);
    or_mooeeinv(vol(L) / 2, Ls, b, c, M5, mf, (double *)te, (double *)te2, dagger);
    or_meo(L, Ls, b, c, M5, mf, U, (double *)te2, 0, (double *)to, dagger);
    or_mooee(vol(L) / 2, Ls, b, c, M5, mf, in_odd, out_odd, dagger);
    cplx *out = (cplx *)out_odd;
    for (long i = 0; i < Nh; i++) out[i] -= to[i];
    free(te); free(te2); free(to);
}

/* ------------------------------------------------------------ vectors */

static double nrm2(long N, const cplx *a)
{
    double s = 0;
#pragma omp parallel for reduction(+ : s) schedule(static)
    for (long i = 0; i < N; i++) s += creal(a[i]) * creal(a[i]) + cimag(a[i]) * cimag(a[i]);
    return s;
}

static cplx dotc(long N, const cplx *a, const cplx *b)
{
    double re = 0, im = 0;
#pragma omp parallel for reduction(+ : re, im) schedule(static)
    for (long i = 0; i < N; i++) {
        cplx t = conj(a[i]) * b[i];
        re += creal(t);
        im += cimag(t);
    }
    return re + I * im;
}

/* ------------------------------------------------------------ CGNE */

typedef struct {
    const int *L; int Ls; double b, c, M5, mf; const double *U;
} ctx_t;

static void mpc_op(const ctx_t *k, const cplx *in, cplx *out, int dagger)
{
    or_mpc(k->L, k->Ls, k->b, k->c, k->M5, k->mf, k->U, (const double *)in, (double *)out, dagger);
}

/* Red-black solve of D5 x = b (full fields):
 *   b~_o = b_o - Moe Mee^-1 b_e
 *   CG on Mpc^+ Mpc x_o = Mpc^+ b~_o from x_o = 0, stop when |r| <= tol |Mpc^+ b~_o|
 *   x_e = Mee^-1 (b_e - Meo x_o)
 * res[0] = normal-equation residual, res[1] = |b~ - Mpc x|/|b~|, res[2] = |b - D5 x|/|b|.
 * x_full on entry holds an initial guess for the odd part when guess != 0.
 * Returns the iteration count, or -iters when maxit was reached. */
int or_cgne(const int *L, int Ls, double b, double c, double M5, double mf, const double *U,
            const double *b_full, double *x_full, double tol, int maxit, int guess, double *res)
{
    ctx_t k = {L, Ls, b, c, M5, mf, U};
    long V = vol(L), Nh = V / 2 * Ls * 12, N = V * Ls * 12;
    cplx *be = malloc(Nh * sizeof(cplx)), *bo = malloc(Nh * sizeof(cplx));
    cplx *t1 = malloc(Nh * sizeof(cplx)), *t2 = malloc(Nh * sizeof(cplx));
    cplx *x = calloc(Nh, sizeof(cplx)), *r = malloc(Nh * sizeof(cplx));
    cplx *p = malloc(Nh * sizeof(cplx)), *Ap = malloc(Nh * sizeof(cplx));
    cplx *bt = malloc(Nh * sizeof(cplx)), *mp = malloc(Nh * sizeof(cplx));
    or_pick(L, Ls, b_full, 0, (double *)be);
    or_pick(L, Ls, b_full, 1, (double *)bo);
    /* b~_o */
    or_mooeeinv(V / 2, Ls, b, c, M5, mf, (double *)be, (double *)t1, 0);
    or_meo(L, Ls, b, c, M5, mf, U, (double *)t1, 0, (double *)t2, 0);
    for (long i = 0; i < Nh; i++) bt[i] = bo[i] - t2[i];
    if (guess) or_pick(L, Ls, x_full, 1, (double *)x);

    /* r = Mpc^+ (b~ - Mpc x) */
    mpc_op(&k, x, t1, 0);
    for (long i = 0; i < Nh; i++) t1[i] = bt[i] - t1[i];
    mpc_op(&k, t1, r, 1);
    mpc_op(&k, bt, t2, 1);
    double rhs2 = nrm2(Nh, t2);
    memcpy(p, r, Nh * sizeof(cplx));
    double rho = nrm2(Nh, r);
    int it = 0, conv = (rho <= tol * tol * rhs2);
    while (!conv && it < maxit) {
        mpc_op(&k, p, mp, 0);
        mpc_op(&k, mp, Ap, 1);
        double pAp = creal(dotc(Nh, p, Ap));
        double alpha = rho / pAp;
        for (long i = 0; i < Nh; i++) {
            x[i] += alpha * p[i];
            r[i] -= alpha * Ap[i];
        }
        double rho1 = nrm2(Nh, r);
        it++;
        if (rho1 <= tol * tol * rhs2) { conv = 1; break; }
        double beta = rho1 / rho;
        for (long i = 0; i < Nh; i++) p[i] = r[i] + beta * p[i];
        rho = rho1;
    }
    /* x_e = Mee^-1 (b_e - Meo x_o) */
    or_meo(L, Ls, b, c, M5, mf, U, (double *)x, 1, (double *)t1, 0);
    for (long i = 0; i < Nh; i++) t1[i] = be[i] - t1[i];
    or_mooeeinv(V / 2, Ls, b, c, M5, mf, (double *)t1, (double *)t2, 0);
    cplx *xf = (cplx *)x_full;
    cplx *tmp = malloc(N * sizeof(cplx));
    or_embed(L, Ls, (double *)t2, 0, (double *)xf);
    or_embed(L, Ls, (double *)x, 1, (double *)tmp);
    for (long i = 0; i < N; i++) xf[i] += tmp[i];
    /* residuals */
    if (res) {
        mpc_op(&k, x, t1, 0);
        for (long i = 0; i < Nh; i++) t1[i] = bt[i] - t1[i];
        res[1] = sqrt(nrm2(Nh, t1) / nrm2(Nh, bt));
        mpc_op(&k, t1, t2, 1);
        res[0] = sqrt(nrm2(Nh, t2) / rhs2);
        or_d5(L, Ls, b, c, M5, mf, U, x_full, (double *)tmp, 0);
        const cplx *bf = (const cplx *)b_full;
        for (long i = 0; i < N; i++) tmp[i] = bf[i] - tmp[i];
        res[2] = sqrt(nrm2(N, tmp) / nrm2(N, bf));
    }
    free(tmp);
    free(be); free(bo); free(t1); free(t2); free(x); free(r); free(p); free(Ap); free(bt); free(mp);
    return conv ? it : -it;
}

/* Red-black source preparation and reconstruction, exposed for the Schur tests. */
void or_schur_source(const int *L, int Ls, double b, double c, double M5, double mf, const double *U,
                     const double *b_full, double *bt_odd)
{
    long V = vol(L), Nh = V / 2 * Ls * 12;
    cplx *be = malloc(Nh * sizeof(cplx)), *bo = malloc(Nh * sizeof(cplx));
    cplx *t1 = malloc(Nh * sizeof(cplx)), *t2 = malloc(Nh * sizeof(cplx));
    or_pick(L, Ls, b_full, 0, (double *)be);
    or_pick(L, Ls, b_full, 1, (double *)bo);
    or_mooeeinv(V / 2, Ls, b, c, M5, mf, (double *)be, (double *)t1, 0);
    or_meo(L, Ls, b, c, M5, mf, U, (double *)t1, 0, (double *)t2, 0);
    cplx *bt = (cplx *)bt_odd;
    for (long i = 0; i < Nh; i++) bt[i] = bo[i] - t2[i];
    free(be); free(bo); free(t1); free(t2);
}

/* ------------------------------------------------------------ multi-shift CG */

/* (Mpc^+ Mpc + sigma_k) x_k = b for every shift, one Krylov space (Jegerlehner).
 * Base system sigma_0 = min sigma.  Shift k is frozen once |zeta_k| |r| <= tol |b|
 * and its zeta is no longer updated.  iters_k returns the iteration at which
 * shift k froze; res_k the true relative residual recomputed at the end.
 * Returns the number of base iterations (negative when maxit was hit). */
int or_multishift(const int *L, int Ls, double b, double c, double M5, double mf, const double *U,
                  const double *b_odd, int nshift, const double *shifts, double *x_odd,
                  double tol, int maxit, int *iters_k, double *res_k)
{
    ctx_t k = {L, Ls, b, c, M5, mf, U};
    long Nh = vol(L) / 2 * Ls * 12;
    const cplx *bb = (const cplx *)b_odd;
    cplx *X = (cplx *)x_odd;
    double s0 = shifts[0];
    for (int j = 1; j < nshift; j++) if (shifts[j] < s0) s0 = shifts[j];
    cplx *r = malloc(Nh * sizeof(cplx)), *Ap = malloc(Nh * sizeof(cplx)), *mp = malloc(Nh * sizeof(cplx));
    cplx *P = malloc((size_t)nshift * Nh * sizeof(cplx));
    double *zeta = malloc(nshift * sizeof(double)), *zeta_old = malloc(nshift * sizeof(double));
    int *active = malloc(nshift * sizeof(int));
    memcpy(r, bb, Nh * sizeof(cplx));
    for (int j = 0; j < nshift; j++) {
        memset(X + (size_t)j * Nh, 0, Nh * sizeof(cplx));
        memcpy(P + (size_t)j * Nh, bb, Nh * sizeof(cplx));
        zeta[j] = zeta_old[j] = 1.0;
        active[j] = 1;
        iters_k[j] = 0;
    }
    double bnorm = sqrt(nrm2(Nh, bb));
    double rho = nrm2(Nh, r);
    double alpha_old = 1.0, beta_old = 0.0;
    /* p (base) is the shift with sigma = s0; keep a separate base direction */
    cplx *p = malloc(Nh * sizeof(cplx));
    memcpy(p, bb, Nh * sizeof(cplx));
    int it = 0, nact = nshift;
    while (nact > 0 && it < maxit) {
        mpc_op(&k, p, mp, 0);
        mpc_op(&k, mp, Ap, 1);
        for (long i = 0; i < Nh; i++) Ap[i] += s0 * p[i];
        double alpha = rho / creal(dotc(Nh, p, Ap));
        for (long i = 0; i < Nh; i++) r[i] -= alpha * Ap[i];
        double rho1 = nrm2(Nh, r);
        double beta = rho1 / rho;
        it++;
        for (int j = 0; j < nshift; j++) {
            if (!active[j]) continue;
            double ds = shifts[j] - s0;
            double z = zeta[j], zo = zeta_old[j];
            double zn = z * zo * alpha_old /
                        (alpha * beta_old * (zo - z) + zo * alpha_old * (1.0 + ds * alpha));
            double as = alpha * zn / z;
            double bs = beta * (zn / z) * (zn / z);
            cplx *x = X + (size_t)j * Nh, *ps = P + (size_t)j * Nh;
            for (long i = 0; i < Nh; i++) x[i] += as * ps[i];
            for (long i = 0; i < Nh; i++) ps[i] = zn * r[i] + bs * ps[i];
            zeta_old[j] = z;
            zeta[j] = zn;
            if (fabs(zn) * sqrt(rho1) <= tol * bnorm) {
                active[j] = 0;
                iters_k[j] = it;
                nact--;
            }
        }
        for (long i = 0; i < Nh; i++) p[i] = r[i] + beta * p[i];
        rho = rho1;
        alpha_old = alpha;
        beta_old = beta;
    }
    for (int j = 0; j < nshift; j++) {
        if (active[j]) iters_k[j] = -it;
        cplx *x = X + (size_t)j * Nh;
        mpc_op(&k, x, mp, 0);
        mpc_op(&k, mp, Ap, 1);
        for (long i = 0; i < Nh; i++) Ap[i] = bb[i] - Ap[i] - shifts[j] * x[i];
        res_k[j] = sqrt(nrm2(Nh, Ap)) / bnorm;
    }
    free(r); free(Ap); free(mp); free(P); free(zeta); free(zeta_old); free(active); free(p);
    return nact ? -it : it;
}

/* ------------------------------------------------------------ PTC network */

/* Parallel-transport convolution layer on the full 5D lattice.
 * Features phi[n][s][chan][colour].  Paths (index pi):
 *   0: identity, 1+mu: U_mu(x) phi(x+mu), 5+mu: U_mu(x-mu)^+ phi(x-mu),
 *   9: phi(x, s+1) (zero at s = Ls-1), 10: phi(x, s-1) (zero at s = 0).
 * Layer: out_a = sum_pi sum_b W[pi][a][b] (T_pi phi_b). */
#define NPATH 11

static void transport(const int *L, int Ls, const cplx *U, int C, const cplx *in, cplx *out, int pi)
{
    long V = vol(L);
#pragma omp parallel for schedule(static)
    for (long n = 0; n < V; n++)
        for (int s = 0; s < Ls; s++)
            for (int ch = 0; ch < C; ch++) {
                cplx *o = out + (((long)n * Ls + s) * C + ch) * 3;
                if (pi == 0) {
                    const cplx *i0 = in + (((long)n * Ls + s) * C + ch) * 3;
                    for (int a = 0; a < 3; a++) o[a] = i0[a];
                } else if (pi <= 4) {
                    int mu = pi - 1;
                    long nf = shifted(L, n, mu, +1);
                    const cplx *i0 = in + (((long)nf * Ls + s) * C + ch) * 3;
                    for (int a = 0; a < 3; a++) {
                        cplx t = 0;
                        for (int bb = 0; bb < 3; bb++) t += U[UIDX(n, mu, a, bb)] * i0[bb];
                        o[a] = t;
                    }
                } else if (pi <= 8) {
                    int mu = pi - 5;
                    long nb = shifted(L, n, mu, -1);
                    const cplx *i0 = in + (((long)nb * Ls + s) * C + ch) * 3;
                    for (int a = 0; a < 3; a++) {
                        cplx t = 0;
                        for (int bb = 0; bb < 3; bb++) t += conj(U[UIDX(nb, mu, bb, a)]) * i0[bb];
                        o[a] = t;
                    }
                } else {
                    int s2 = (pi == 9) ? s + 1 : s - 1;
                    if (s2 < 0 || s2 >= Ls) {
                        for (int a = 0; a < 3; a++) o[a] = 0;
                    } else {
                        const cplx *i0 = in + (((long)n * Ls + s2) * C + ch) * 3;
                        for (int a = 0; a < 3; a++) o[a] = i0[a];
                    }
                }
            }
}

/* adjoint path of pi: (T_{+mu})^+ = T_{-mu}, (T_{+s})^+ = T_{-s} */
static int adjoint_path(int pi)
{
    if (pi == 0) return 0;
    if (pi <= 4) return pi + 4;
    if (pi <= 8) return pi - 4;
    return (pi == 9) ? 10 : 9;
}

/* one layer: W[pi][a][b] complex, shape (11, Cout, Cin) */
void or_ptc_layer(const int *L, int Ls, const double *U_, int Cin, int Cout, const double *W_,
                  const double *in_, double *out_)
{
    const cplx *U = (const cplx *)U_, *W = (const cplx *)W_, *in = (const cplx *)in_;
    cplx *out = (cplx *)out_;
    long V5 = vol(L) * Ls;
    cplx *T = malloc(V5 * Cin * 3 * sizeof(cplx));
    memset(out, 0, V5 * Cout * 3 * sizeof(cplx));
    for (int pi = 0; pi < NPATH; pi++) {
        transport(L, Ls, U, Cin, in, T, pi);
#pragma omp parallel for schedule(static)
        for (long i = 0; i < V5; i++)
            for (int a = 0; a < Cout; a++)
                for (int cc = 0; cc < 3; cc++) {
                    cplx t = 0;
                    for (int bb = 0; bb < Cin; bb++) t += W[((long)pi * Cout + a) * Cin + bb] * T[(i * Cin + bb) * 3 + cc];
                    out[(i * Cout + a) * 3 + cc] += t;
                }
    }
    free(T);
}

/* Backward of one layer.  g_out holds 2 dL/d conj(out) (the real-pair gradient
 * dL/dRe + i dL/dIm).  Produces g_in = 2 dL/d conj(in) = sum_pi T_pi^+ W_pi^+ g_out
 * and accumulates g_W[pi][a][b] += sum_{x,s,c} g_out_a conj(T_pi in_b), the same
 * real-pair gradient for the weights. */
void or_ptc_layer_backward(const int *L, int Ls, const double *U_, int Cin, int Cout, const double *W_,
                           const double *in_, const double *gout_, double *gin_, double *gW_)
{
    const cplx *U = (const cplx *)U_, *W = (const cplx *)W_, *in = (const cplx *)in_;
    const cplx *gout = (const cplx *)gout_;
    cplx *gin = (cplx *)gin_, *gW = (cplx *)gW_;
    long V5 = vol(L) * Ls;
    cplx *T = malloc(V5 * (Cin > Cout ? Cin : Cout) * 3 * sizeof(cplx));
    cplx *Y = malloc(V5 * Cin * 3 * sizeof(cplx));
    if (gin) memset(gin, 0, V5 * Cin * 3 * sizeof(cplx));
    for (int pi = 0; pi < NPATH; pi++) {
        /* weight gradient */
        if (gW) {
            transport(L, Ls, U, Cin, in, T, pi);
            for (int a = 0; a < Cout; a++)
                for (int bb = 0; bb < Cin; bb++) {
                    double re = 0, im = 0;
#pragma omp parallel for reduction(+ : re, im) schedule(static)
                    for (long i = 0; i < V5; i++)
                        for (int cc = 0; cc < 3; cc++) {
                            cplx t = gout[(i * Cout + a) * 3 + cc] * conj(T[(i * Cin + bb) * 3 + cc]);
                            re += creal(t);
                            im += cimag(t);
                        }
                    gW[((long)pi * Cout + a) * Cin + bb] += re + I * im;
                }
        }
        /* input gradient: Y_b = sum_a conj(W_ab) g_a, then T_pi^+ Y */
        if (gin) {
#pragma omp parallel for schedule(static)
            for (long i = 0; i < V5; i++)
                for (int bb = 0; bb < Cin; bb++)
                    for (int cc = 0; cc < 3; cc++) {
                        cplx t = 0;
                        for (int a = 0; a < Cout; a++) t += conj(W[((long)pi * Cout + a) * Cin + bb]) * gout[(i * Cout + a) * 3 + cc];
                        Y[(i * Cin + bb) * 3 + cc] = t;
                    }
            transport(L, Ls, U, Cin, Y, T, adjoint_path(pi));
            for (long i = 0; i < V5 * Cin * 3; i++) gin[i] += T[i];
        }
    }
    free(T);
    free(Y);
}

/* -------------------------------------------------------------- FGCR */

/* Network preconditioner for the odd Schur system: embed the odd residual
 * (spin components as 4 channels) into the full lattice with zeros on even
 * sites, run the layers, restrict the 4 output channels to odd sites.
 * chans has nlayer+1 entries; W holds the layers' (11, Cout, Cin) blocks back to back. */
void or_net_apply(const int *L, int Ls, const double *U, int nlayer, const int *chans, const double *W_,
                  const double *in_odd, double *out_odd)
{
    const cplx *W = (const cplx *)W_;
    long V5 = vol(L) * Ls;
    int cmax = 0;
    for (int l = 0; l <= nlayer; l++) if (chans[l] > cmax) cmax = chans[l];
    cplx *a = malloc(V5 * cmax * 3 * sizeof(cplx));
    cplx *bq = malloc(V5 * cmax * 3 * sizeof(cplx));
    /* [n][s][spin][colour] is exactly [n][s][chan=spin][colour] */
    or_embed(L, Ls, in_odd, 1, (double *)a);
    long off = 0;
    for (int l = 0; l < nlayer; l++) {
        or_ptc_layer(L, Ls, U, chans[l], chans[l + 1], (const double *)(W + off), (double *)a, (double *)bq);
        off += (long)NPATH * chans[l] * chans[l + 1];
        cplx *t = a; a = bq; bq = t;
    }
    or_pick(L, Ls, (double *)a, 1, out_odd);
    free(a);
    free(bq);
}

/* Flexible GCR(m) on A x = b over odd sites, right-preconditioned by the
 * network (nlayer = 0: no preconditioner, plain GCR).  A = Mpc (normal = 0) or
 * A = Mpc^+ Mpc (normal = 1).  Restart every m steps with the residual
 * recomputed.  Returns iterations (negative on maxit). */
static void fgcr_op(const ctx_t *k, const cplx *in, cplx *out, cplx *tmp, int normal)
{
    if (normal) {
        mpc_op(k, in, tmp, 0);
        mpc_op(k, tmp, out, 1);
    } else {
        mpc_op(k, in, out, 0);
    }
}

int or_fgcr(const int *L, int Ls, double b, double c, double M5, double mf, const double *U,
            int nlayer, const int *chans, const double *W, const double *b_odd, double *x_odd,
            double tol, int maxit, int m, int normal, double *res)
{
    ctx_t k = {L, Ls, b, c, M5, mf, U};
    long Nh = vol(L) / 2 * Ls * 12;
    const cplx *bb = (const cplx *)b_odd;
    cplx *x = (cplx *)x_odd;
    cplx *r = malloc(Nh * sizeof(cplx));
    cplx *Z = malloc((size_t)m * Nh * sizeof(cplx)), *Q = malloc((size_t)m * Nh * sizeof(cplx));
    cplx *tmp = malloc(Nh * sizeof(cplx));
    memset(x, 0, Nh * sizeof(cplx));
    memcpy(r, bb, Nh * sizeof(cplx));
    double bn = sqrt(nrm2(Nh, bb));
    int it = 0, conv = 0;
    while (!conv && it < maxit) {
        for (int kk = 0; kk < m && it < maxit; kk++) {
            cplx *z = Z + (size_t)kk * Nh, *q = Q + (size_t)kk * Nh;
            if (nlayer > 0) or_net_apply(L, Ls, U, nlayer, chans, W, (double *)r, (double *)z);
            else memcpy(z, r, Nh * sizeof(cplx));
            fgcr_op(&k, z, q, tmp, normal);
            for (int j = 0; j < kk; j++) {
                cplx *qj = Q + (size_t)j * Nh, *zj = Z + (size_t)j * Nh;
                cplx be = dotc(Nh, qj, q);
                for (long i = 0; i < Nh; i++) { q[i] -= be * qj[i]; z[i] -= be * zj[i]; }
            }
            double qn = sqrt(nrm2(Nh, q));
            for (long i = 0; i < Nh; i++) { q[i] /= qn; z[i] /= qn; }
            cplx al = dotc(Nh, q, r);
            for (long i = 0; i < Nh; i++) { x[i] += al * z[i]; r[i] -= al * q[i]; }
            it++;
            if (sqrt(nrm2(Nh, r)) <= tol * bn) break;
        }
        /* restart / final check with the true residual */
        fgcr_op(&k, x, r, tmp, normal);
        for (long i = 0; i < Nh; i++) r[i] = bb[i] - r[i];
        if (sqrt(nrm2(Nh, r)) <= tol * bn) conv = 1;
    }
    if (res) res[0] = sqrt(nrm2(Nh, r)) / bn;
    free(r); free(Z); free(Q); free(tmp);
    return conv ? it : -it;
}
