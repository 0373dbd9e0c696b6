/*
 * mw_oracle.c -- plain FP64 CPU reference for the McEwen-Wiaux (MW) spin
 * spherical-harmonic transforms (McEwen & Wiaux, "A novel sampling theorem on
 * the sphere", IEEE TSP 59(12), 2011).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code, header, table or constant generator
 * with the GPU path.
 *
 * Every stage is written the slow, obvious way, in the paper's order and
 * notation:
 *   - Delta^l_{m,n} = d^l_{mn}(pi/2) from Risbo's half-step recursion
 *     (the method the paper uses for its timings, Sec. V-B/V-C; the recursion
 *     itself is from Risbo, J. Geodesy 1996, not printed in the paper),
 *   - every Fourier sum is a direct O(N^2) DFT with exactly reduced angles,
 *   - the weight convolution is the direct Toeplitz sum of Eq.(Gmm_convolution),
 *   - the contractions are Eq.(flm_wig) and Eq.(Fmm) summed over the full
 *     m' range, with no symmetry folding.
 * OpenMP parallelises independent outputs only; the arithmetic of each output
 * is sequential in a fixed order.
 *
 * Layouts (all complex values are interleaved re,im doubles = C99 double complex):
 *   map   f[t*(2L-1) + p],  t < L (theta_t = pi(2t+1)/(2L-1)), p < 2L-1
 *   coeff flm[l*l + l + m], 0 <= l < L, |m| <= l  (entries with l < |s| are 0)
 *   planes indexed by m + (L-1) for |m| <= L-1.
 * Return value: 0 on success, -1 on bad arguments, -2 on allocation failure.
 */
#include <complex.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef double complex cplx;

static const double PI = 3.14159265358979323846264338327950288;

void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* exp(-2 pi i k / N) for an integer k reduced exactly modulo N. */
static cplx unit_root(long long k, long long N)
{
    long long r = k % N;
    if (r < 0) r += N;
    double a = 2.0 * PI * (double)r / (double)N;
    return cos(a) - I * sin(a);
}

/* i^k for integer k. */
static cplx ipow(int k)
{
    int r = ((k % 4) + 4) % 4;
    if (r == 0) return 1.0;
    if (r == 1) return I;
    if (r == 2) return -1.0;
    return -I;
}

static double sgn(int k) { return (k % 2 == 0) ? 1.0 : -1.0; }

/* ------------------------------------------------------------------------ */
/* Wigner Delta planes by Risbo's recursion.                                  */
/*                                                                           */
/* A plane of order j (j integer or half-integer, stored as twoj = 2j) holds */
/* d^j_{mn}(pi/2) at [a][b], a = m + j, b = n + j, a,b in [0, 2j].            */
/* One half-step j-1/2 -> j couples each entry to its four neighbours in     */
/* the previous plane through the Clebsch-Gordan weights of spin 1/2,        */
/*   cp(a) = sqrt(a/2j),  cm(a) = sqrt((2j-a)/2j),                           */
/* and the spin-1/2 rotation by beta = pi/2,                                 */
/*   u = [[cos(b/2), -sin(b/2)], [sin(b/2), cos(b/2)]] = [[1,-1],[1,1]]/sqrt2. */
/* Two half-steps advance l by one.                                          */
/* ------------------------------------------------------------------------ */
typedef struct {
    int twoj;      /* 2j of the plane currently held in cur */
    int stride;    /* row stride: planes carry a zero border of width 1 */
    double *cur, *nxt;
    double *cp, *cm;
} risbo_t;

/* Entry (a, b) of a plane, a, b in [-1, 2j+1] (the border entries stay zero). */
#define RAT(buf, R, a, b) ((buf)[(size_t)((a) + 1) * (size_t)(R)->stride + (size_t)((b) + 1)])

static int risbo_init(risbo_t* R, int lmax)
{
    R->stride = 2 * lmax + 3;
    size_t n = (size_t)R->stride * (size_t)R->stride;
    R->cur = (double*)calloc(n, sizeof(double));
    R->nxt = (double*)calloc(n, sizeof(double));
    R->cp = (double*)calloc((size_t)R->stride + 1, sizeof(double));
    R->cm = (double*)calloc((size_t)R->stride + 1, sizeof(double));
    if (!R->cur || !R->nxt || !R->cp || !R->cm) return -2;
    R->twoj = 0;
    RAT(R->cur, R, 0, 0) = 1.0; /* d^0_{00} = 1 */
    return 0;
}

static void risbo_free(risbo_t* R)
{
    free(R->cur); free(R->nxt); free(R->cp); free(R->cm);
}

/* Planes only grow, so every entry outside the current plane (including the
 * border row/column -1) is zero in both buffers. */
static void risbo_halfstep(risbo_t* R)
{
    const int tj = R->twoj + 1; /* 2j of the new plane */
    const double r = 1.0 / sqrt(2.0);
    for (int a = 0; a <= tj; ++a) {
        R->cp[a] = sqrt((double)a / (double)tj);
        R->cm[a] = sqrt((double)(tj - a) / (double)tj);
    }
    const double* P = R->cur;
    double* Q = R->nxt;
    #pragma omp parallel for schedule(static)
    for (int a = 0; a <= tj; ++a) {
        for (int b = 0; b <= tj; ++b) {
            double v = R->cp[a] * R->cp[b] * RAT(P, R, a - 1, b - 1)
                     - R->cp[a] * R->cm[b] * RAT(P, R, a - 1, b)
                     + R->cm[a] * R->cp[b] * RAT(P, R, a, b - 1)
                     + R->cm[a] * R->cm[b] * RAT(P, R, a, b);
            RAT(Q, R, a, b) = r * v;
        }
    }
    double* t = R->cur; R->cur = R->nxt; R->nxt = t;
    R->twoj = tj;
}

/* Advance to integer order l (must be >= current order). */
static void risbo_to(risbo_t* R, int l)
{
    while (R->twoj < 2 * l) risbo_halfstep(R);
}

/* Delta^l_{m,n} from a plane of integer order l. */
static double D(const risbo_t* R, int l, int m, int n)
{
    return RAT(R->cur, R, m + l, n + l);
}

int orc_delta_plane(int l, double* out)
{
    if (l < 0 || !out) return -1;
    risbo_t R;
    if (risbo_init(&R, l)) { risbo_free(&R); return -2; }
    risbo_to(&R, l);
    for (int m = -l; m <= l; ++m)
        for (int n = -l; n <= l; ++n) out[(size_t)(m + l) * (2 * l + 1) + (n + l)] = D(&R, l, m, n);
    risbo_free(&R);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Harmonic weights (Sec. IV-D, weights of Eq.(Gmm_convolution)):            */
/*   w(k) = +-i pi/2 for k = +-1, 0 for other odd k, 2/(1-k^2) for even k.    */
/* ------------------------------------------------------------------------ */
static cplx weight(int k)
{
    if (k == 1) return I * PI / 2.0;
    if (k == -1) return -I * PI / 2.0;
    if (k % 2 != 0) return 0.0;
    return 2.0 / (1.0 - (double)k * (double)k);
}

void orc_weights(int L, double* out_ri)
{
    /* w(k) for k = -2(L-1) .. 2(L-1) */
    cplx* o = (cplx*)out_ri;
    for (int k = -2 * (L - 1); k <= 2 * (L - 1); ++k) o[k + 2 * (L - 1)] = weight(k);
}

static int check_args(int L, int s)
{
    if (L < 1 || L > 8192) return -1;
    if (s <= -L || s >= L) return -1;
    return 0;
}

/* ======================================================================== */
/* Forward transform, stage by stage (Sec. IV-D, algorithm Forward Transform) */
/* ======================================================================== */

/* Stage 1, phi-DFT: G_m(theta_t) = 2pi/(2L-1) sum_p f(theta_t, phi_p) e^{-i m phi_p},
 * phi_p = 2 pi p/(2L-1).  Output Gtm[t][m + L-1], t < L. */
static void fwd_phi(int L, const cplx* f, cplx* Gtm)
{
    const int N1 = 2 * L - 1;
    #pragma omp parallel for collapse(2) schedule(static)
    for (int t = 0; t < L; ++t)
        for (int m = -(L - 1); m <= L - 1; ++m) {
            cplx acc = 0.0;
            for (int p = 0; p < N1; ++p)
                acc += f[(size_t)t * N1 + p] * unit_root((long long)m * p, N1);
            Gtm[(size_t)t * N1 + (m + L - 1)] = (2.0 * PI / N1) * acc;
        }
}

/* Stage 2, periodic extension in theta (Sec. IV-B/IV-D):
 *   Gext_m(theta_t) = G_m(theta_t) for t < L,
 *   Gext_m(theta_t) = (-1)^{m+s} G_m(theta_{2L-2-t}) for L <= t <= 2L-2. */
static void fwd_extend(int L, int s, const cplx* Gtm, cplx* Gext)
{
    const int N1 = 2 * L - 1;
    for (int t = 0; t < N1; ++t)
        for (int m = -(L - 1); m <= L - 1; ++m) {
            cplx v;
            if (t < L) v = Gtm[(size_t)t * N1 + (m + L - 1)];
            else v = sgn(m + s) * Gtm[(size_t)(2 * L - 2 - t) * N1 + (m + L - 1)];
            Gext[(size_t)t * N1 + (m + L - 1)] = v;
        }
}

/* Stage 3, theta-DFT: F_{m m'} = 1/(2 pi (2L-1)) sum_{t=0}^{2L-2} Gext_m(theta_t) e^{-i m' theta_t},
 * theta_t = pi (2t+1)/(2L-1), i.e. e^{-i m' theta_t} = exp(-2 pi i m'(2t+1)/(2(2L-1))).
 * Output F[m][m'] (both offset by L-1). */
static void fwd_theta(int L, const cplx* Gext, cplx* F)
{
    const int N1 = 2 * L - 1;
    #pragma omp parallel for collapse(2) schedule(static)
    for (int m = -(L - 1); m <= L - 1; ++m)
        for (int mp = -(L - 1); mp <= L - 1; ++mp) {
            cplx acc = 0.0;
            for (int t = 0; t < N1; ++t)
                acc += Gext[(size_t)t * N1 + (m + L - 1)] *
                       unit_root((long long)mp * (2 * t + 1), 2LL * N1);
            F[(size_t)(m + L - 1) * N1 + (mp + L - 1)] = acc / (2.0 * PI * N1);
        }
}

/* Stage 4, weight convolution, Eq.(Gmm_convolution):
 *   G_{m m'} = 2 pi sum_{m''=-(L-1)}^{L-1} F_{m m''} w(m'' - m'). */
static void fwd_weights(int L, const cplx* F, cplx* Gmm)
{
    const int N1 = 2 * L - 1;
    #pragma omp parallel for collapse(2) schedule(static)
    for (int m = -(L - 1); m <= L - 1; ++m)
        for (int mp = -(L - 1); mp <= L - 1; ++mp) {
            cplx acc = 0.0;
            for (int mpp = -(L - 1); mpp <= L - 1; ++mpp)
                acc += F[(size_t)(m + L - 1) * N1 + (mpp + L - 1)] * weight(mpp - mp);
            Gmm[(size_t)(m + L - 1) * N1 + (mp + L - 1)] = 2.0 * PI * acc;
        }
}

/* Stage 5, Eq.(flm_wig):
 *   f_lm = (-1)^s i^{m+s} sqrt((2l+1)/4pi) sum_{m'=-l}^{l} Delta^l_{m' m} Delta^l_{m',-s} G_{m m'}.
 * Coefficients with l < |s| are left zero. When ms != NULL only the listed
 * orders m are produced (out[k][l] for ms[k]); otherwise flm is filled. */
static int fwd_contract(int L, int s, const cplx* Gmm, cplx* flm, int nm, const int* ms, cplx* out)
{
    const int N1 = 2 * L - 1;
    risbo_t R;
    if (risbo_init(&R, L - 1)) { risbo_free(&R); return -2; }
    if (flm) memset(flm, 0, sizeof(cplx) * (size_t)L * L);
    if (out) memset(out, 0, sizeof(cplx) * (size_t)nm * L);
    for (int l = 0; l < L; ++l) {
        risbo_to(&R, l);
        if (l < abs(s)) continue;
        const double nl = sqrt((2.0 * l + 1.0) / (4.0 * PI));
        if (!ms) {
            #pragma omp parallel for schedule(static)
            for (int m = -l; m <= l; ++m) {
                cplx acc = 0.0;
                for (int mp = -l; mp <= l; ++mp)
                    acc += D(&R, l, mp, m) * D(&R, l, mp, -s) * Gmm[(size_t)(m + L - 1) * N1 + (mp + L - 1)];
                flm[(size_t)l * l + l + m] = sgn(s) * ipow(m + s) * nl * acc;
            }
        } else {
            #pragma omp parallel for schedule(static)
            for (int k = 0; k < nm; ++k) {
                int m = ms[k];
                if (m < -l || m > l) continue;
                cplx acc = 0.0;
                for (int mp = -l; mp <= l; ++mp)
                    acc += D(&R, l, mp, m) * D(&R, l, mp, -s) * Gmm[(size_t)(m + L - 1) * N1 + (mp + L - 1)];
                out[(size_t)k * L + l] = sgn(s) * ipow(m + s) * nl * acc;
            }
        }
    }
    risbo_free(&R);
    return 0;
}

int orc_forward_stages(int L, int s, const double* f_ri, double* Gtm_ri, double* F_ri,
                       double* Gmm_ri, double* flm_ri)
{
    if (check_args(L, s) || !f_ri) return -1;
    const int N1 = 2 * L - 1;
    const cplx* f = (const cplx*)f_ri;
    cplx* Gtm = (cplx*)malloc(sizeof(cplx) * (size_t)L * N1);
    cplx* Gext = (cplx*)malloc(sizeof(cplx) * (size_t)N1 * N1);
    cplx* F = (cplx*)malloc(sizeof(cplx) * (size_t)N1 * N1);
    cplx* Gmm = (cplx*)malloc(sizeof(cplx) * (size_t)N1 * N1);
    int rc = 0;
    if (!Gtm || !Gext || !F || !Gmm) { rc = -2; goto done; }
    fwd_phi(L, f, Gtm);
    fwd_extend(L, s, Gtm, Gext);
    fwd_theta(L, Gext, F);
    fwd_weights(L, F, Gmm);
    if (Gtm_ri) memcpy(Gtm_ri, Gtm, sizeof(cplx) * (size_t)L * N1);
    if (F_ri) memcpy(F_ri, F, sizeof(cplx) * (size_t)N1 * N1);
    if (Gmm_ri) memcpy(Gmm_ri, Gmm, sizeof(cplx) * (size_t)N1 * N1);
    if (flm_ri) rc = fwd_contract(L, s, Gmm, (cplx*)flm_ri, 0, NULL, NULL);
done:
    free(Gtm); free(Gext); free(F); free(Gmm);
    return rc;
}

int orc_forward(int L, int s, const double* f_ri, double* flm_ri)
{
    if (!flm_ri) return -1;
    return orc_forward_stages(L, s, f_ri, NULL, NULL, NULL, flm_ri);
}

/* Forward transform restricted to the listed orders: out[k][l] = f_{l, ms[k]}
 * (zero where |ms[k]| > l).  Stages 1-4 are evaluated for those m only. */
int orc_forward_orders(int L, int s, const double* f_ri, int nm, const int* ms, double* out_ri)
{
    if (check_args(L, s) || !f_ri || nm < 1 || !ms || !out_ri) return -1;
    const int N1 = 2 * L - 1;
    for (int k = 0; k < nm; ++k) if (ms[k] <= -L || ms[k] >= L) return -1;
    const cplx* f = (const cplx*)f_ri;
    cplx* Gmm = (cplx*)calloc((size_t)N1 * N1, sizeof(cplx));
    cplx* Gm = (cplx*)malloc(sizeof(cplx) * (size_t)N1);  /* extended column */
    cplx* Fm = (cplx*)malloc(sizeof(cplx) * (size_t)N1);
    int rc = 0;
    if (!Gmm || !Gm || !Fm) { rc = -2; goto done; }
    for (int k = 0; k < nm; ++k) {
        const int m = ms[k];
        /* stage 1 for this m, all rings */
        #pragma omp parallel for schedule(static)
        for (int t = 0; t < L; ++t) {
            cplx acc = 0.0;
            for (int p = 0; p < N1; ++p)
                acc += f[(size_t)t * N1 + p] * unit_root((long long)m * p, N1);
            Gm[t] = (2.0 * PI / N1) * acc;
        }
        /* stage 2 */
        for (int t = L; t < N1; ++t) Gm[t] = sgn(m + s) * Gm[2 * L - 2 - t];
        /* stage 3 */
        #pragma omp parallel for schedule(static)
        for (int mp = -(L - 1); mp <= L - 1; ++mp) {
            cplx acc = 0.0;
            for (int t = 0; t < N1; ++t) acc += Gm[t] * unit_root((long long)mp * (2 * t + 1), 2LL * N1);
            Fm[mp + L - 1] = acc / (2.0 * PI * N1);
        }
        /* stage 4 */
        #pragma omp parallel for schedule(static)
        for (int mp = -(L - 1); mp <= L - 1; ++mp) {
            cplx acc = 0.0;
            for (int mpp = -(L - 1); mpp <= L - 1; ++mpp) acc += Fm[mpp + L - 1] * weight(mpp - mp);
            Gmm[(size_t)(m + L - 1) * N1 + (mp + L - 1)] = 2.0 * PI * acc;
        }
    }
    rc = fwd_contract(L, s, Gmm, NULL, nm, ms, (cplx*)out_ri);
done:
    free(Gmm); free(Gm); free(Fm);
    return rc;
}

/* ======================================================================== */
/* Inverse transform (Sec. IV-E, algorithm Inverse Transform)                 */
/* ======================================================================== */

/* Step 1, Eq.(Fmm):
 *   F_{m m'} = (-1)^s i^{-(m+s)} sum_{l} sqrt((2l+1)/4pi) Delta^l_{m' m} Delta^l_{m',-s} f_lm,
 * for all |m|, |m'| <= L-1, l from max(|m|,|m'|,|s|) to L-1. */
static int inv_contract(int L, int s, const cplx* flm, cplx* F)
{
    const int N1 = 2 * L - 1;
    risbo_t R;
    if (risbo_init(&R, L - 1)) { risbo_free(&R); return -2; }
    memset(F, 0, sizeof(cplx) * (size_t)N1 * N1);
    for (int l = 0; l < L; ++l) {
        risbo_to(&R, l);
        if (l < abs(s)) continue;
        const double nl = sqrt((2.0 * l + 1.0) / (4.0 * PI));
        #pragma omp parallel for collapse(2) schedule(static)
        for (int m = -l; m <= l; ++m)
            for (int mp = -l; mp <= l; ++mp)
                F[(size_t)(m + L - 1) * N1 + (mp + L - 1)] +=
                    nl * D(&R, l, mp, m) * D(&R, l, mp, -s) * flm[(size_t)l * l + l + m];
    }
    for (int m = -(L - 1); m <= L - 1; ++m)
        for (int mp = -(L - 1); mp <= L - 1; ++mp)
            F[(size_t)(m + L - 1) * N1 + (mp + L - 1)] *= sgn(s) * ipow(-(m + s));
    risbo_free(&R);
    return 0;
}

/* Step 2, Eq.(Fmt): F_m(theta_t) = sum_{m'} F_{m m'} e^{i m' theta_t}, evaluated
 * for t < L only (the samples on (pi, 2pi) are discarded).  Output Fmt[m][t]. */
static void inv_theta(int L, const cplx* F, cplx* Fmt)
{
    const int N1 = 2 * L - 1;
    #pragma omp parallel for collapse(2) schedule(static)
    for (int m = -(L - 1); m <= L - 1; ++m)
        for (int t = 0; t < L; ++t) {
            cplx acc = 0.0;
            for (int mp = -(L - 1); mp <= L - 1; ++mp)
                acc += F[(size_t)(m + L - 1) * N1 + (mp + L - 1)] *
                       conj(unit_root((long long)mp * (2 * t + 1), 2LL * N1));
            Fmt[(size_t)(m + L - 1) * L + t] = acc;
        }
}

/* Step 3, Eq.(f_pfft): f(theta_t, phi_p) = sum_m F_m(theta_t) e^{i m phi_p}. */
static void inv_phi(int L, const cplx* Fmt, cplx* f)
{
    const int N1 = 2 * L - 1;
    #pragma omp parallel for collapse(2) schedule(static)
    for (int t = 0; t < L; ++t)
        for (int p = 0; p < N1; ++p) {
            cplx acc = 0.0;
            for (int m = -(L - 1); m <= L - 1; ++m)
                acc += Fmt[(size_t)(m + L - 1) * L + t] * conj(unit_root((long long)m * p, N1));
            f[(size_t)t * N1 + p] = acc;
        }
}

int orc_inverse_stages(int L, int s, const double* flm_ri, double* F_ri, double* Fmt_ri, double* f_ri)
{
    if (check_args(L, s) || !flm_ri) return -1;
    const int N1 = 2 * L - 1;
    cplx* F = (cplx*)malloc(sizeof(cplx) * (size_t)N1 * N1);
    cplx* Fmt = (cplx*)malloc(sizeof(cplx) * (size_t)N1 * L);
    int rc = 0;
    if (!F || !Fmt) { rc = -2; goto done; }
    rc = inv_contract(L, s, (const cplx*)flm_ri, F);
    if (rc) goto done;
    inv_theta(L, F, Fmt);
    if (F_ri) memcpy(F_ri, F, sizeof(cplx) * (size_t)N1 * N1);
    if (Fmt_ri) memcpy(Fmt_ri, Fmt, sizeof(cplx) * (size_t)N1 * L);
    if (f_ri) inv_phi(L, Fmt, (cplx*)f_ri);
done:
    free(F); free(Fmt);
    return rc;
}

/* Inverse restricted to the listed orders: out[k][t] = F_{ms[k]}(theta_t), t < L,
 * i.e. Eq.(Fmm) for those m followed by Eq.(Fmt); equal to the phi-Fourier
 * coefficient of ring t of the inverse map at order ms[k]. */
int orc_inverse_orders(int L, int s, const double* flm_ri, int nm, const int* ms, double* out_ri)
{
    if (check_args(L, s) || !flm_ri || nm < 1 || !ms || !out_ri) return -1;
    const int N1 = 2 * L - 1;
    for (int k = 0; k < nm; ++k) if (ms[k] <= -L || ms[k] >= L) return -1;
    const cplx* flm = (const cplx*)flm_ri;
    cplx* out = (cplx*)out_ri;
    cplx* F = (cplx*)calloc((size_t)nm * N1, sizeof(cplx));
    risbo_t R;
    int rc = risbo_init(&R, L - 1);
    if (rc || !F) { rc = -2; goto done; }
    for (int l = 0; l < L; ++l) {
        risbo_to(&R, l);
        if (l < abs(s)) continue;
        const double nl = sqrt((2.0 * l + 1.0) / (4.0 * PI));
        #pragma omp parallel for schedule(static)
        for (int k = 0; k < nm; ++k) {
            const int m = ms[k];
            if (m < -l || m > l) continue;
            for (int mp = -l; mp <= l; ++mp)
                F[(size_t)k * N1 + (mp + L - 1)] += nl * D(&R, l, mp, m) * D(&R, l, mp, -s) * flm[(size_t)l * l + l + m];
        }
    }
    #pragma omp parallel for collapse(2) schedule(static)
    for (int k = 0; k < nm; ++k)
        for (int t = 0; t < L; ++t) {
            const int m = ms[k];
            cplx acc = 0.0;
            for (int mp = -(L - 1); mp <= L - 1; ++mp)
                acc += sgn(s) * ipow(-(m + s)) * F[(size_t)k * N1 + (mp + L - 1)] *
                       conj(unit_root((long long)mp * (2 * t + 1), 2LL * N1));
            out[(size_t)k * L + t] = acc;
        }
done:
    risbo_free(&R);
    free(F);
    return rc;
}

int orc_inverse(int L, int s, const double* flm_ri, double* f_ri)
{
    if (!f_ri) return -1;
    return orc_inverse_stages(L, s, flm_ri, NULL, NULL, f_ri);
}

/* ======================================================================== */
/* Adjoints with respect to the plain Euclidean inner products on the full   */
/* L x (2L-1) grid and on the L^2 coefficients.  Each is the conjugate        */
/* transpose of the stages above, applied in reverse order.                   */
/* ======================================================================== */

/* A^H for the forward map: coefficients y_lm -> grid. */
int orc_forward_adjoint(int L, int s, const double* y_ri, double* f_ri)
{
    if (check_args(L, s) || !y_ri || !f_ri) return -1;
    const int N1 = 2 * L - 1;
    const cplx* y = (const cplx*)y_ri;
    cplx* f = (cplx*)f_ri;
    cplx* Y = (cplx*)calloc((size_t)N1 * N1, sizeof(cplx));
    cplx* Z = (cplx*)malloc(sizeof(cplx) * (size_t)N1 * N1);
    cplx* Gext = (cplx*)malloc(sizeof(cplx) * (size_t)N1 * N1);
    cplx* Gtm = (cplx*)malloc(sizeof(cplx) * (size_t)L * N1);
    risbo_t R;
    int rc = risbo_init(&R, L - 1);
    if (rc || !Y || !Z || !Gext || !Gtm) { rc = -2; goto done; }
    /* stage 5^H: Y_{m m'} = sum_l conj(c_lm) Delta^l_{m'm} Delta^l_{m',-s} y_lm */
    for (int l = 0; l < L; ++l) {
        risbo_to(&R, l);
        if (l < abs(s)) continue;
        const double nl = sqrt((2.0 * l + 1.0) / (4.0 * PI));
        #pragma omp parallel for collapse(2) schedule(static)
        for (int m = -l; m <= l; ++m)
            for (int mp = -l; mp <= l; ++mp)
                Y[(size_t)(m + L - 1) * N1 + (mp + L - 1)] +=
                    conj(sgn(s) * ipow(m + s) * nl) * D(&R, l, mp, m) * D(&R, l, mp, -s) *
                    y[(size_t)l * l + l + m];
    }
    /* stage 4^H: Z_{m m''} = 2 pi sum_{m'} conj(w(m''-m')) Y_{m m'} */
    #pragma omp parallel for collapse(2) schedule(static)
    for (int m = -(L - 1); m <= L - 1; ++m)
        for (int mpp = -(L - 1); mpp <= L - 1; ++mpp) {
            cplx acc = 0.0;
            for (int mp = -(L - 1); mp <= L - 1; ++mp)
                acc += conj(weight(mpp - mp)) * Y[(size_t)(m + L - 1) * N1 + (mp + L - 1)];
            Z[(size_t)(m + L - 1) * N1 + (mpp + L - 1)] = 2.0 * PI * acc;
        }
    /* stage 3^H: Gext_m(theta_t) = 1/(2 pi N1) sum_{m'} e^{+i m' theta_t} Z_{m m'} */
    #pragma omp parallel for collapse(2) schedule(static)
    for (int t = 0; t < N1; ++t)
        for (int m = -(L - 1); m <= L - 1; ++m) {
            cplx acc = 0.0;
            for (int mp = -(L - 1); mp <= L - 1; ++mp)
                acc += conj(unit_root((long long)mp * (2 * t + 1), 2LL * N1)) *
                       Z[(size_t)(m + L - 1) * N1 + (mp + L - 1)];
            Gext[(size_t)t * N1 + (m + L - 1)] = acc / (2.0 * PI * N1);
        }
    /* stage 2^H: fold the extension back onto t < L */
    for (int t = 0; t < L; ++t)
        for (int m = -(L - 1); m <= L - 1; ++m) {
            cplx v = Gext[(size_t)t * N1 + (m + L - 1)];
            if (t <= L - 2) v += sgn(m + s) * Gext[(size_t)(2 * L - 2 - t) * N1 + (m + L - 1)];
            Gtm[(size_t)t * N1 + (m + L - 1)] = v;
        }
    /* stage 1^H: f(t, p) = 2pi/N1 sum_m e^{+i m phi_p} G_m(theta_t) */
    #pragma omp parallel for collapse(2) schedule(static)
    for (int t = 0; t < L; ++t)
        for (int p = 0; p < N1; ++p) {
            cplx acc = 0.0;
            for (int m = -(L - 1); m <= L - 1; ++m)
                acc += conj(unit_root((long long)m * p, N1)) * Gtm[(size_t)t * N1 + (m + L - 1)];
            f[(size_t)t * N1 + p] = (2.0 * PI / N1) * acc;
        }
done:
    risbo_free(&R);
    free(Y); free(Z); free(Gext); free(Gtm);
    return rc;
}

/* Y^H for the inverse map: grid g -> coefficients. */
int orc_inverse_adjoint(int L, int s, const double* g_ri, double* y_ri)
{
    if (check_args(L, s) || !g_ri || !y_ri) return -1;
    const int N1 = 2 * L - 1;
    const cplx* g = (const cplx*)g_ri;
    cplx* y = (cplx*)y_ri;
    cplx* X = (cplx*)malloc(sizeof(cplx) * (size_t)L * N1);
    cplx* Z = (cplx*)malloc(sizeof(cplx) * (size_t)N1 * N1);
    risbo_t R;
    int rc = risbo_init(&R, L - 1);
    if (rc || !X || !Z) { rc = -2; goto done; }
    /* step 3^H: X_m(t) = sum_p e^{-i m phi_p} g(t, p) */
    #pragma omp parallel for collapse(2) schedule(static)
    for (int t = 0; t < L; ++t)
        for (int m = -(L - 1); m <= L - 1; ++m) {
            cplx acc = 0.0;
            for (int p = 0; p < N1; ++p) acc += unit_root((long long)m * p, N1) * g[(size_t)t * N1 + p];
            X[(size_t)t * N1 + (m + L - 1)] = acc;
        }
    /* step 2^H: Z_{m m'} = sum_{t<L} e^{-i m' theta_t} X_m(t) */
    #pragma omp parallel for collapse(2) schedule(static)
    for (int m = -(L - 1); m <= L - 1; ++m)
        for (int mp = -(L - 1); mp <= L - 1; ++mp) {
            cplx acc = 0.0;
            for (int t = 0; t < L; ++t)
                acc += unit_root((long long)mp * (2 * t + 1), 2LL * N1) * X[(size_t)t * N1 + (m + L - 1)];
            Z[(size_t)(m + L - 1) * N1 + (mp + L - 1)] = acc;
        }
    /* step 1^H: y_lm = sum_{m'} conj((-1)^s i^{-(m+s)}) sqrt((2l+1)/4pi) Delta Delta Z_{m m'} */
    memset(y, 0, sizeof(cplx) * (size_t)L * L);
    for (int l = 0; l < L; ++l) {
        risbo_to(&R, l);
        if (l < abs(s)) continue;
        const double nl = sqrt((2.0 * l + 1.0) / (4.0 * PI));
        #pragma omp parallel for schedule(static)
        for (int m = -l; m <= l; ++m) {
            cplx acc = 0.0;
            for (int mp = -l; mp <= l; ++mp)
                acc += D(&R, l, mp, m) * D(&R, l, mp, -s) * Z[(size_t)(m + L - 1) * N1 + (mp + L - 1)];
            y[(size_t)l * l + l + m] = conj(sgn(s) * ipow(-(m + s))) * nl * acc;
        }
    }
done:
    risbo_free(&R);
    free(X); free(Z);
    return rc;
}

/* ======================================================================== */
/* Row recursion in the second index at beta = pi/2 (the Trapani-Navaza      */
/* family the paper compares with Risbo, Sec. V-C), in plain FP64 from the    */
/* edge value Delta^l_{m,l} = 2^{-l} sqrt(binom(2l, l+m)).  Used only to      */
/* reproduce the paper's observation that this kind of recursion loses        */
/* accuracy at very large l when run without exponent extension.             */
/*   sqrt((l+n)(l-n+1)) Delta_{m,n-1} = -2m Delta_{m,n} - sqrt((l-n)(l+n+1)) Delta_{m,n+1} */
/* out[n] = Delta^l_{m,n} for n = 0..l.                                        */
/* ======================================================================== */
int orc_row_plain(int l, int m, double* out)
{
    if (l < 0 || m < 0 || m > l || !out) return -1;
    double e = 1.0;
    for (int k = 1; k <= l; ++k) e *= sqrt((2.0 * k - 1.0) / (2.0 * k)); /* Delta^l_{0,l} */
    for (int k = 1; k <= m; ++k) e *= sqrt((double)(l - k + 1) / (double)(l + k));
    double dn = e, dn1 = 0.0;
    out[l] = dn;
    for (int n = l; n >= 1; --n) {
        double an = sqrt((double)(l + n) * (double)(l - n + 1));
        double an1 = sqrt((double)(l - n) * (double)(l + n + 1));
        double dm1 = -(2.0 * m * dn + an1 * dn1) / an;
        dn1 = dn; dn = dm1;
        out[n - 1] = dn;
    }
    return 0;
}

/* ======================================================================== */
/* Explicit quadrature (Sec. IV-F, Eq.(quadrature)).                          */
/* ======================================================================== */
/* wtilde(theta_t) = 1/(2L-1) sum_{m'=-(L-1)}^{L-1} w(-m') e^{i m' theta_t}
 * (the inverse DFT of the reflected weights), and the weights
 *   q(theta_t) = (2 pi/L) [wtilde(theta_t) + (1 - delta_{t,L-1}) (-1)^s wtilde(theta_{2L-2-t})],
 * t < L (the contributions of (pi, 2 pi) folded back onto [0, pi]).
 * q_ri[2t], q_ri[2t+1] = Re, Im of q(theta_t); the imaginary part vanishes up
 * to rounding (w(-m') and w(m') are conjugate). */
static cplx wtilde(int L, int t)
{
    const int N1 = 2 * L - 1;
    cplx acc = 0.0;
    for (int mp = -(L - 1); mp <= L - 1; ++mp)
        acc += weight(-mp) * conj(unit_root((long long)mp * (2 * t + 1), 2LL * N1));
    return acc / (double)N1;
}

int orc_quad_weights(int L, int s, double* q_ri)
{
    if (check_args(L, s) || !q_ri) return -1;
    cplx* q = (cplx*)q_ri;
    for (int t = 0; t < L; ++t) {
        cplx v = wtilde(L, t);
        if (t != L - 1) v += sgn(s) * wtilde(L, 2 * L - 2 - t);
        q[t] = (2.0 * PI / L) * v;
    }
    return 0;
}

/* I = sum_{t<L} sum_{p<nphi} f(theta_t, 2 pi p/nphi) q(theta_t) (L/nphi).
 * nphi = L is the paper's rule (phi'_p = 2 pi p/L, L(L-1)+1 distinct samples);
 * nphi = 2L-1 applies the same theta weights on the transform grid, the phi
 * sum (2 pi/nphi) sum_p being the exact phi integral of a band-limited ring for
 * either nphi.  f: [t][p] complex, L x nphi.  out_ri: Re, Im of I. */
int orc_integrate(int L, int s, int nphi, const double* f_ri, double* out_ri)
{
    if (check_args(L, s) || (nphi != L && nphi != 2 * L - 1) || !f_ri || !out_ri) return -1;
    const cplx* f = (const cplx*)f_ri;
    cplx* q = (cplx*)malloc(sizeof(cplx) * (size_t)L);
    if (!q) return -2;
    orc_quad_weights(L, s, (double*)q);
    cplx acc = 0.0;
    for (int t = 0; t < L; ++t) {
        cplx ring = 0.0;
        for (int p = 0; p < nphi; ++p) ring += f[(size_t)t * nphi + p];
        acc += ring * creal(q[t]);
    }
    *(cplx*)out_ri = acc * ((double)L / (double)nphi);
    free(q);
    return 0;
}
