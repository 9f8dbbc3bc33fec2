/*
 * mcdi_oracle.c -- plain, slow, FP64 CPU oracle for the differentiable Monte
 * Carlo direct-illumination estimator of Hasselgren, Hofmann & Munkberg,
 * "Shape, Light, and Material Decomposition from Images using Monte Carlo
 * Rendering and Denoising" (NeurIPS 2022).
 *
 * TEST INFRASTRUCTURE.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load this file.  It shares no code, header,
 * table or constant generator with the HIP library; the only thing both sides
 * consume is the seeded synthetic input.
 *
 * What it computes, in the paper's order (section 3.1 "Direct Illumination",
 * section 4.1 "Multiple Importance Sampling", appendix A "Optimization and
 * Regularization" for the visibility term H, appendix D "Sampling"):
 *   - the rendering equation restricted to direct light from an environment
 *     probe, estimated by Monte Carlo with shadow rays (section 3.1);
 *   - three sampling techniques combined with the balance heuristic: a
 *     piecewise-constant 2D distribution over the probe, cosine sampling of the
 *     diffuse lobe and visible-normal sampling of the GGX lobe (section 4.1);
 *   - detached sampling and detached visibility: gradients flow only through
 *     the material evaluation (section 3.1 "Shadow gradients", section 4.1);
 *   - the same random numbers are replayed in the backward pass (section 4.1,
 *     appendix D);
 *   - diffuse lighting is returned demodulated, specular is not (section 4.2);
 *   - shadowed samples are weighted by H = 1 - tau (appendix A); the
 *     incident radiance is the probe's times H, so with H = 0 a blocked
 *     direction carries none, whatever the probe holds there (also where it
 *     is not finite, where an IEEE product would give NaN);
 *   - separately, the visibility gradient that the estimator detaches: the
 *     derivative of the shadowed integral with respect to the occluding mesh's
 *     vertices (section 3.1 "Shadow gradients"; appendix "Visibility
 *     Gradients from Shadows"), estimated by sampling silhouette edges.
 * Points the paper leaves open (probe parameterisation, lobe selection
 * probability, GGX details, ray offsets, RNG) take one reading each, stated
 * where the code implements it, and the kernels take the same.
 *
 * Everything here is FP64 except two discrete decisions that the HIP kernel
 * takes in FP32 and that the oracle therefore also takes in FP32: the
 * lobe-selection probability q and the roughness clamp.  The probe's sampling
 * tables are FP64 sums rounded once to FP32, because the tables themselves are
 * an output that both sides must agree on bit for bit.
 *
 * Parity unpinned: nothing; every function is pinned by a test against a
 * closed form, a library routine, a quadrature or a brute-force evaluation.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Counter-based RNG: Philox4x32-10 (Salmon, Moraes, Dror, Shaw; SC 2011).   */
/* Ten rounds of two 32x32->64 multiplies and a key schedule (Weyl sequence).*/
/* ------------------------------------------------------------------------ */
void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 24 high bits of a 32-bit word as a uniform number in [0, 1). Exact. */
static double u01(uint32_t x) { return (double)(x >> 8) * (1.0 / 16777216.0); }

/* The eight uniforms of sample s of a pixel: two Philox blocks keyed by the
 * 64-bit seed, with counter (pixel in view, global view id, s, block). */
static void sample_uniforms(uint64_t seed, uint32_t pix_in_view, uint32_t view_id,
                            uint32_t s, double xi[8])
{
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    uint32_t c[4] = {pix_in_view, view_id, s, 0u}, o[4];
    orc_philox4x32_10(c, key, o);
    for (int k = 0; k < 4; ++k) xi[k] = u01(o[k]);
    c[3] = 1u;
    orc_philox4x32_10(c, key, o);
    for (int k = 0; k < 4; ++k) xi[4 + k] = u01(o[k]);
}

/* ------------------------------------------------------------------------ */
/* Piecewise-constant 2D distribution over the lat-long probe (section 4.1,  */
/* appendix D: light importance sampling).  Row i covers polar angle         */
/* [i, i+1) * pi/H measured from +Y, column j covers azimuth [j, j+1)*2pi/W. */
/* Texel weight = luminance (r+g+b)/3 (clamped at 0) times sin(theta) at the */
/* row centre.                                                               */
/* ------------------------------------------------------------------------ */
static double texel_weight(const float* env, int W, int i, int j, double sin_row)
{
    const float* t = env + ((size_t)i * W + j) * 3;
    double y = ((double)t[0] + (double)t[1] + (double)t[2]) / 3.0;
    if (!(y > 0.0) || !isfinite(y)) y = 0.0;
    return y * sin_row;
}

/* Tables: cond [H][W+1] (per-row CDF), marg [H+1] (marginal CDF over rows),
 * pdf [H][W] = (w_ij / sum w) * W * H, the density in (u, v) of texel (i,j).
 * Sums run left to right in FP64; each entry is rounded once to FP32.
 * Returns 1 if the total weight is positive (light sampling enabled). */
int orc_env_tables(const float* env, int H, int W, float* cond, float* marg, float* pdf,
                   double* total_out)
{
    double* rowsum = (double*)malloc(sizeof(double) * (size_t)H);
    for (int i = 0; i < H; ++i) {
        double srow = sin(ORC_PI * ((double)i + 0.5) / (double)H);
        double run = 0.0;
        for (int j = 0; j < W; ++j) run += texel_weight(env, W, i, j, srow);
        rowsum[i] = run;
        float* c = cond + (size_t)i * (W + 1);
        double prefix = 0.0;
        c[0] = 0.0f;
        for (int j = 0; j + 1 < W; ++j) {
            prefix += texel_weight(env, W, i, j, srow);
            c[j + 1] = run > 0.0 ? (float)(prefix / run) : (float)((double)(j + 1) / (double)W);
        }
        c[W] = 1.0f;
    }
    double total = 0.0;
    for (int i = 0; i < H; ++i) total += rowsum[i];
    double prefix = 0.0;
    marg[0] = 0.0f;
    for (int i = 0; i + 1 < H; ++i) {
        prefix += rowsum[i];
        marg[i + 1] = total > 0.0 ? (float)(prefix / total) : (float)((double)(i + 1) / (double)H);
    }
    marg[H] = 1.0f;
    for (int i = 0; i < H; ++i) {
        double srow = sin(ORC_PI * ((double)i + 0.5) / (double)H);
        for (int j = 0; j < W; ++j) {
            double w = texel_weight(env, W, i, j, srow);
            pdf[(size_t)i * W + j] = total > 0.0 ? (float)((w / total) * ((double)W * (double)H)) : 0.0f;
        }
    }
    free(rowsum);
    if (total_out) *total_out = total;
    return total > 0.0;
}

/* Largest k in [0, n-1] with cdf[k] <= x (cdf[0] = 0 <= x < 1 = cdf[n]).
 * Zero-width bins are skipped because a later equal entry also qualifies. */
static int cdf_search(const float* cdf, int n, double x)
{
    int k = 0;
    for (int i = 1; i < n; ++i)
        if ((double)cdf[i] <= x) k = i;
    return k;
}

typedef struct {
    int32_t H, W;
    const float* env;   /* [H][W][3] radiance used for shading */
    const float* cond;  /* [H][W+1] */
    const float* marg;  /* [H+1] */
    const float* pdf;   /* [H][W] */
    int32_t light_enabled;
} orc_env;

/* Direction of (u, v) in [0,1)^2: theta = pi v from +Y, phi = 2 pi u. */
static void dir_of_uv(double u, double v, double w[3])
{
    double th = ORC_PI * v, ph = 2.0 * ORC_PI * u;
    w[0] = sin(th) * cos(ph);
    w[1] = cos(th);
    w[2] = sin(th) * sin(ph);
}

/* Sample the probe: returns texel (i, j), the direction, its solid-angle
 * density p = pdf_uv / (2 pi^2 sin theta) and the continuous texel
 * coordinates (x, y) = (u W, v H) of the sample. */
static void sample_light_xy(const orc_env* e, double xi0, double xi1, double w[3], double* p,
                            int32_t* ti, int32_t* tj, double* x, double* y)
{
    int H = e->H, W = e->W;
    int i = cdf_search(e->marg, H, xi0);
    const float* c = e->cond + (size_t)i * (W + 1);
    int j = cdf_search(c, W, xi1);
    double dv = (xi0 - (double)e->marg[i]) / ((double)e->marg[i + 1] - (double)e->marg[i]);
    double du = (xi1 - (double)c[j]) / ((double)c[j + 1] - (double)c[j]);
    double v = ((double)i + dv) / (double)H, u = ((double)j + du) / (double)W;
    dir_of_uv(u, v, w);
    double st = sin(ORC_PI * v);
    *p = st > 0.0 ? (double)e->pdf[(size_t)i * W + j] / (2.0 * ORC_PI * ORC_PI * st) : 0.0;
    *ti = i;
    *tj = j;
    *x = (double)j + du;
    *y = (double)i + dv;
}

void orc_sample_light(const orc_env* e, double xi0, double xi1, double w[3], double* p,
                      int32_t* ti, int32_t* tj)
{
    double x, y;
    sample_light_xy(e, xi0, xi1, w, p, ti, tj, &x, &y);
}

/* Texel of a unit direction (nearest lookup) and the angular distance, in
 * radians of arc, to the closest texel boundary that would change it. */
static void texel_of_dir_xy(int H, int W, const double w[3], int* ti, int* tj, double* margin,
                            double* x, double* y)
{
    double rho = sqrt(w[0] * w[0] + w[2] * w[2]);
    double th = atan2(rho, w[1]);
    double ph = atan2(w[2], w[0]);
    if (ph < 0.0) ph += 2.0 * ORC_PI;
    double fi = th * (double)H / ORC_PI, fj = ph * (double)W / (2.0 * ORC_PI);
    int i = (int)floor(fi), j = (int)floor(fj);
    if (i > H - 1) i = H - 1;
    if (i < 0) i = 0;
    if (j > W - 1) j = W - 1;
    if (j < 0) j = 0;
    double m = INFINITY;
    /* interior row boundaries 1..H-1 */
    double ri = floor(fi + 0.5);
    if (ri >= 1.0 && ri <= (double)(H - 1)) m = fmin(m, fabs(fi - ri) * ORC_PI / (double)H);
    /* column boundaries 0..W (0 and W are the same seam) */
    double rj = floor(fj + 0.5);
    m = fmin(m, fabs(fj - rj) * 2.0 * ORC_PI / (double)W * rho);
    *ti = i;
    *tj = j;
    *margin = m;
    if (x) *x = fj;
    if (y) *y = fi;
}

static void texel_of_dir(int H, int W, const double w[3], int* ti, int* tj, double* margin)
{
    texel_of_dir_xy(H, W, w, ti, tj, margin, NULL, NULL);
}

/* ------------------------------------------------------------------------ */
/* Bilinear probe reconstruction.  Section 3.1 stores the probe as a float   */
/* texture without naming the lookup filter; the default reading is the     */
/* nearest texel, this is the filtered one.  The light technique keeps the  */
/* piecewise-constant density of the texels either way (section 4.1).       */
/* ------------------------------------------------------------------------ */

/* Tent weight of integer tap k at coordinate s (texel centres at integers). */
static double tent(double s, int k)
{
    double d = fabs(s - (double)k);
    return d < 1.0 ? 1.0 - d : 0.0;
}

static int wrap_col(int j, int W) { j %= W; return j < 0 ? j + W : j; }
static int clamp_row(int i, int H) { return i < 0 ? 0 : (i > H - 1 ? H - 1 : i); }

static const float* texel_ptr(const float* env, int H, int W, int i, int j)
{
    return env + ((size_t)clamp_row(i, H) * W + wrap_col(j, W)) * 3;
}

/* Radiance at continuous texel coordinates (x, y) = (phi W / 2 pi, theta H /
 * pi): texel (i, j) covers [j, j+1) x [i, i+1) and its value sits at the
 * centre (j + 1/2, i + 1/2).  The reconstruction is the sum over texels of
 * tent(x - 1/2, j) tent(y - 1/2, i) env[i][j], with columns wrapping across
 * the phi = 0 seam and rows clamped at the poles; the weights sum to one. */
void orc_probe_bilinear(const float* env, int H, int W, double x, double y, double L[3])
{
    double xs = x - 0.5, ys = y - 0.5;
    int j0 = (int)floor(xs), i0 = (int)floor(ys);
    for (int c = 0; c < 3; ++c) L[c] = 0.0;
    for (int i = i0; i <= i0 + 1; ++i)
        for (int j = j0; j <= j0 + 1; ++j) {
            double wt = tent(ys, i) * tent(xs, j);
            const float* e = texel_ptr(env, H, W, i, j);
            for (int c = 0; c < 3; ++c) L[c] += wt * (double)e[c];
        }
}

/* Bound, per channel, on how far an FP32 reconstruction can be from this one
 * when (x, y) move by at most (dx, dy).  Inside one cell the reconstruction
 * is bilinear in the offsets, so the change is exactly Lx ex + Ly ey + Lxy ex
 * ey for offsets (ex, ey): bounded by |Lx| dx + |Ly| dy + |Lxy| dx dy.  Where
 * the move can leave the cell, the largest neighbouring-texel difference in
 * the 4x4 neighbourhood bounds the slope (beyond one texel: twice the largest
 * magnitude in the rows the move can reach).  Plus the FP32 rounding of the
 * tap weights and of the four-tap sum: a few units in the last place of the
 * sum of the taps' magnitudes. */
static void bilinear_shift_bound(const float* env, int H, int W, double x, double y, double dx,
                                 double dy, double dL[3])
{
    const double xs = x - 0.5, ys = y - 0.5;
    const int j0 = (int)floor(xs), i0 = (int)floor(ys);
    const double fx = xs - j0, fy = ys - i0;
    const int inside = fx >= dx && fx + dx <= 1.0 && fy >= dy && fy + dy <= 1.0;
    for (int c = 0; c < 3; ++c) {
        const double aa = texel_ptr(env, H, W, i0, j0)[c], ab = texel_ptr(env, H, W, i0, j0 + 1)[c];
        const double ba = texel_ptr(env, H, W, i0 + 1, j0)[c], bb = texel_ptr(env, H, W, i0 + 1, j0 + 1)[c];
        const double r = 8.0 * 0x1p-24 * (fabs(aa) + fabs(ab) + fabs(ba) + fabs(bb));
        if (inside) {
            const double Lx = (1.0 - fy) * (ab - aa) + fy * (bb - ba);
            const double Ly = (1.0 - fx) * (ba - aa) + fx * (bb - ab);
            const double Lxy = bb - ba - ab + aa;
            dL[c] = fabs(Lx) * dx + fabs(Ly) * dy + fabs(Lxy) * dx * dy + r;
            continue;
        }
        if (dx >= 1.0 || dy >= 1.0) {
            int rr = (int)ceil(dy) + 1;
            double mx = 0.0;
            for (int i = i0 - rr; i <= i0 + 1 + rr; ++i)
                for (int j = 0; j < W; ++j) mx = fmax(mx, fabs((double)texel_ptr(env, H, W, i, j)[c]));
            dL[c] = 2.0 * mx + r;
            continue;
        }
        double sx = 0.0, sy = 0.0;
        for (int i = i0 - 1; i <= i0 + 2; ++i)
            for (int j = j0 - 1; j <= j0 + 2; ++j) {
                double e = texel_ptr(env, H, W, i, j)[c];
                sx = fmax(sx, fabs(e - (double)texel_ptr(env, H, W, i, j - 1)[c]));
                sy = fmax(sy, fabs(e - (double)texel_ptr(env, H, W, i - 1, j)[c]));
            }
        dL[c] = dx * sx + dy * sy + r;
    }
}

/* Solid-angle density of the light technique at a direction. */
double orc_pdf_light(const orc_env* e, const double w[3])
{
    if (!e->light_enabled) return 0.0;
    int i, j;
    double m;
    texel_of_dir(e->H, e->W, w, &i, &j, &m);
    double rho = sqrt(w[0] * w[0] + w[2] * w[2]);
    return rho > 0.0 ? (double)e->pdf[(size_t)i * e->W + j] / (2.0 * ORC_PI * ORC_PI * rho) : 0.0;
}

/* ------------------------------------------------------------------------ */
/* Vectors                                                                    */
/* ------------------------------------------------------------------------ */
static double dot3(const double a[3], const double b[3]) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double a[3], const double b[3], double c[3])
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double a[3]) { return sqrt(dot3(a, a)); }

/* Orthonormal basis (t, b) around unit n, branch-free construction of Duff
 * et al. (JCGT 2017).  `sgn` is the sign of n_z as given by the caller. */
static void onb(const double n[3], double sgn, double t[3], double b[3])
{
    double a = -1.0 / (sgn + n[2]);
    double bb = n[0] * n[1] * a;
    t[0] = 1.0 + sgn * n[0] * n[0] * a;
    t[1] = sgn * bb;
    t[2] = -sgn * n[0];
    b[0] = bb;
    b[1] = sgn + n[1] * n[1] * a;
    b[2] = -n[1];
}

/* ------------------------------------------------------------------------ */
/* Material model (section 3): a diffuse term plus an isotropic GGX specular */
/* lobe (Walter et al. 2007).  alpha = roughness^2, Smith height-correlated  */
/* masking-shadowing, Schlick Fresnel with F0 = lerp(0.04, kd, metallic).    */
/* ------------------------------------------------------------------------ */

/* GGX normal distribution written with s2 = |n x h|^2 for 1 - (n.h)^2. */
double orc_ggx_D(double noh, double s2, double alpha)
{
    if (!(noh > 0.0)) return 0.0;
    double a2 = alpha * alpha;
    double den = a2 * noh * noh + s2;
    return a2 / (ORC_PI * den * den);
}

/* Smith Lambda for GGX at cos = x > 0. */
double orc_ggx_lambda(double x, double alpha)
{
    double t2 = (1.0 - x * x) / (x * x);
    return 0.5 * (-1.0 + sqrt(1.0 + alpha * alpha * t2));
}

static double lambda_dalpha(double x, double alpha)
{
    double t2 = (1.0 - x * x) / (x * x);
    return alpha * t2 / (2.0 * sqrt(1.0 + alpha * alpha * t2));
}

static double lambda_dx(double x, double alpha)
{
    double a2 = alpha * alpha;
    return -a2 / (2.0 * x * x * x * sqrt(1.0 + a2 * (1.0 / (x * x) - 1.0)));
}

/* Density of visible-normal sampling after reflection about h (Heitz 2018):
 * G1(wo) D(h) / (4 n.wo), in local coordinates (z = normal). */
double orc_pdf_ggx_local(const double V[3], const double L[3], double alpha)
{
    if (!(V[2] > 0.0)) return 0.0;
    double h[3] = {V[0] + L[0], V[1] + L[1], V[2] + L[2]};
    double hl = norm3(h);
    if (!(hl > 0.0)) return 0.0;
    for (int k = 0; k < 3; ++k) h[k] /= hl;
    double s2 = h[0] * h[0] + h[1] * h[1];
    double D = orc_ggx_D(h[2], s2, alpha);
    double G1 = 1.0 / (1.0 + orc_ggx_lambda(V[2], alpha));
    return G1 * D / (4.0 * V[2]);
}

double orc_pdf_cos_local(const double L[3]) { return L[2] > 0.0 ? L[2] / ORC_PI : 0.0; }

/* Cosine-weighted hemisphere sample, polar mapping. */
void orc_sample_cos_local(double u1, double u2, double L[3])
{
    double r = sqrt(u1), ph = 2.0 * ORC_PI * u2;
    L[0] = r * cos(ph);
    L[1] = r * sin(ph);
    L[2] = sqrt(fmax(0.0, 1.0 - u1));
}

/* Intermediates of one visible-normal sample that decide how much FP32
 * roundoff its direction can carry: g = 1 - t1^2 and h = 1 - t1^2 - t2^2 (the
 * arguments of the two square roots), the blend weight s and the length of
 * the un-stretched normal before normalisation. */
typedef struct {
    double g, h, s, mlen;
} vndf_aux;

/* Visible-normal sampling of GGX (Heitz, JCGT 2018): stretch the view vector,
 * sample the projected visible hemisphere, un-stretch the normal, reflect.
 * Returns lensq of the stretched view's tangential part (the degenerate-frame
 * decision); aux (may be NULL) receives the intermediates above. */
static double sample_vndf_aux(const double V[3], double alpha, double u1, double u2, double L[3], vndf_aux* aux)
{
    double vh[3] = {alpha * V[0], alpha * V[1], V[2]};
    double l = norm3(vh);
    for (int k = 0; k < 3; ++k) vh[k] /= l;
    double lensq = vh[0] * vh[0] + vh[1] * vh[1];
    double T1[3], T2[3];
    if (lensq > 0.0) {
        double il = 1.0 / sqrt(lensq);
        T1[0] = -vh[1] * il;
        T1[1] = vh[0] * il;
        T1[2] = 0.0;
    } else {
        T1[0] = 1.0; T1[1] = 0.0; T1[2] = 0.0;
    }
    cross3(vh, T1, T2);
    double r = sqrt(u1), ph = 2.0 * ORC_PI * u2;
    double t1 = r * cos(ph), t2 = r * sin(ph);
    double s = 0.5 * (1.0 + vh[2]);
    const double g = 1.0 - t1 * t1;
    t2 = (1.0 - s) * sqrt(fmax(0.0, g)) + s * t2;
    const double h = 1.0 - t1 * t1 - t2 * t2;
    double tz = sqrt(fmax(0.0, h));
    double nh[3];
    for (int k = 0; k < 3; ++k) nh[k] = t1 * T1[k] + t2 * T2[k] + tz * vh[k];
    double ne[3] = {alpha * nh[0], alpha * nh[1], fmax(0.0, nh[2])};
    double nl = norm3(ne);
    for (int k = 0; k < 3; ++k) ne[k] /= nl;
    double vn = dot3(V, ne);
    for (int k = 0; k < 3; ++k) L[k] = 2.0 * vn * ne[k] - V[k];
    if (aux) {
        aux->g = g;
        aux->h = h;
        aux->s = s;
        aux->mlen = nl;
    }
    return lensq;
}

double orc_sample_vndf_local(const double V[3], double alpha, double u1, double u2, double L[3])
{
    return sample_vndf_aux(V, alpha, u1, u2, L, NULL);
}

/* ------------------------------------------------------------------------ */
/* Shadow-ray visibility (section 3.1): any triangle hit along the ray from  */
/* o in direction d, t in (0, inf), no back-face culling.  Evaluated in FP64 */
/* with a margin: each answer is classified as robust (every ray within the  */
/* tolerance gives the same answer) or undecided.                            */
/* ------------------------------------------------------------------------ */
typedef struct {
    double lo[3], hi[3];
    int32_t left, right; /* children, -1 for a leaf */
    int32_t start, count;
} onode;

typedef struct {
    int64_t ntri;
    double* v;        /* [ntri][9] vertex coordinates */
    int32_t* order;   /* triangle order in leaves */
    onode* nodes;
    int64_t nnodes;
    double center[3];
    double diag;
} orc_scene;

static void tri_bounds(const double* t, double lo[3], double hi[3])
{
    for (int k = 0; k < 3; ++k) {
        lo[k] = fmin(t[k], fmin(t[3 + k], t[6 + k]));
        hi[k] = fmax(t[k], fmax(t[3 + k], t[6 + k]));
    }
}

static double centroid(const double* t, int axis) { return (t[axis] + t[3 + axis] + t[6 + axis]) / 3.0; }

/* Median-free object partition at the midpoint of the centroid bounds along
 * the longest axis; a range that cannot be split that way is cut in half. */
static int32_t build_node(orc_scene* s, int32_t start, int32_t count)
{
    int32_t id = (int32_t)s->nnodes++;
    onode* nd = &s->nodes[id];
    double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int k = 0; k < 3; ++k) { nd->lo[k] = INFINITY; nd->hi[k] = -INFINITY; }
    for (int32_t q = start; q < start + count; ++q) {
        const double* t = s->v + (size_t)s->order[q] * 9;
        double lo[3], hi[3];
        tri_bounds(t, lo, hi);
        for (int k = 0; k < 3; ++k) {
            nd->lo[k] = fmin(nd->lo[k], lo[k]);
            nd->hi[k] = fmax(nd->hi[k], hi[k]);
            double c = centroid(t, k);
            clo[k] = fmin(clo[k], c);
            chi[k] = fmax(chi[k], c);
        }
    }
    if (count <= 4) {
        nd->left = nd->right = -1;
        nd->start = start;
        nd->count = count;
        return id;
    }
    int axis = 0;
    for (int k = 1; k < 3; ++k)
        if (chi[k] - clo[k] > chi[axis] - clo[axis]) axis = k;
    double mid = 0.5 * (clo[axis] + chi[axis]);
    int32_t i = start, j = start + count - 1;
    while (i <= j) {
        if (centroid(s->v + (size_t)s->order[i] * 9, axis) < mid) {
            ++i;
        } else {
            int32_t tmp = s->order[i];
            s->order[i] = s->order[j];
            s->order[j] = tmp;
            --j;
        }
    }
    int32_t nleft = i - start;
    if (nleft == 0 || nleft == count) nleft = count / 2;
    int32_t l = build_node(s, start, nleft);
    int32_t r = build_node(s, start + nleft, count - nleft);
    nd = &s->nodes[id];
    nd->left = l;
    nd->right = r;
    nd->start = start;
    nd->count = 0;
    return id;
}

orc_scene* orc_scene_build(const float* verts, int64_t nv, const int32_t* tris, int64_t nt)
{
    orc_scene* s = (orc_scene*)calloc(1, sizeof(orc_scene));
    s->ntri = nt;
    s->v = (double*)malloc(sizeof(double) * 9 * (size_t)(nt > 0 ? nt : 1));
    s->order = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nt > 0 ? nt : 1));
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t f = 0; f < nt; ++f) {
        for (int c = 0; c < 3; ++c) {
            int32_t vi = tris[f * 3 + c];
            for (int k = 0; k < 3; ++k) {
                double x = (vi >= 0 && vi < nv) ? (double)verts[(size_t)vi * 3 + k] : 0.0;
                s->v[f * 9 + c * 3 + k] = x;
                lo[k] = fmin(lo[k], x);
                hi[k] = fmax(hi[k], x);
            }
        }
        s->order[f] = (int32_t)f;
    }
    double d2 = 0.0;
    for (int k = 0; k < 3; ++k) {
        s->center[k] = nt > 0 ? 0.5 * (lo[k] + hi[k]) : 0.0;
        d2 += nt > 0 ? (hi[k] - lo[k]) * (hi[k] - lo[k]) : 0.0;
    }
    s->diag = sqrt(d2);
    s->nodes = (onode*)malloc(sizeof(onode) * (size_t)(2 * (nt > 0 ? nt : 1)));
    s->nnodes = 0;
    if (nt > 0) build_node(s, 0, (int32_t)nt);
    return s;
}

void orc_scene_free(orc_scene* s)
{
    if (!s) return;
    free(s->v);
    free(s->order);
    free(s->nodes);
    free(s);
}

enum { TRI_MISS = 0, TRI_HIT = 1, TRI_NEAR = 2 };

/* Distance from the 2D origin to segment a-b. */
static double seg_dist(const double a[2], const double b[2])
{
    double ab[2] = {b[0] - a[0], b[1] - a[1]};
    double l2 = ab[0] * ab[0] + ab[1] * ab[1];
    double t = l2 > 0.0 ? -(a[0] * ab[0] + a[1] * ab[1]) / l2 : 0.0;
    if (t < 0.0) t = 0.0;
    if (t > 1.0) t = 1.0;
    double x = a[0] + t * ab[0], y = a[1] + t * ab[1];
    return sqrt(x * x + y * y);
}

/* Classify one triangle against the ray (o, d) with basis (e1, e2) spanning
 * the plane orthogonal to d.  Vertices are projected on that plane; the ray
 * hits iff the origin lies inside the projected triangle and the hit
 * distance along d is positive.  delta_abs/delta_rel give the tolerance. */
static int classify_tri(const double* tv, const double o[3], const double d[3],
                        const double e1[3], const double e2[3], double delta_abs, double delta_rel)
{
    double P[3][2], tk[3];
    double tmaxabs = 0.0;
    for (int c = 0; c < 3; ++c) {
        double q[3] = {tv[c * 3] - o[0], tv[c * 3 + 1] - o[1], tv[c * 3 + 2] - o[2]};
        P[c][0] = dot3(q, e1);
        P[c][1] = dot3(q, e2);
        tk[c] = dot3(q, d);
        tmaxabs = fmax(tmaxabs, fabs(tk[c]));
    }
    double delta = delta_abs + delta_rel * tmaxabs;
    double E0 = P[1][0] * P[2][1] - P[1][1] * P[2][0];
    double E1 = P[2][0] * P[0][1] - P[2][1] * P[0][0];
    double E2 = P[0][0] * P[1][1] - P[0][1] * P[1][0];
    double A = E0 + E1 + E2;
    int inside = (A > 0.0 && E0 > 0.0 && E1 > 0.0 && E2 > 0.0) ||
                 (A < 0.0 && E0 < 0.0 && E1 < 0.0 && E2 < 0.0);
    double bd = fmin(seg_dist(P[0], P[1]), fmin(seg_dist(P[1], P[2]), seg_dist(P[2], P[0])));
    double tmax = fmax(tk[0], fmax(tk[1], tk[2]));
    if (inside && bd > delta) {
        double t = (E0 * tk[0] + E1 * tk[1] + E2 * tk[2]) / A;
        if (t > delta) return TRI_HIT;
        if (t < -delta) return TRI_MISS;
        return TRI_NEAR;
    }
    if (!inside && bd > delta) return TRI_MISS;
    if (tmax < -delta) return TRI_MISS;
    return TRI_NEAR;
}

/* Does the whole line o + t d (any t) meet the box grown by pad?  The line,
 * not the ray, so that the candidate set covers every triangle the
 * classification can call hit or undecided. */
static int box_hit_padded(const onode* nd, const double o[3], const double d[3], double pad)
{
    double t0 = -INFINITY, t1 = INFINITY;
    for (int k = 0; k < 3; ++k) {
        double lo = nd->lo[k] - pad, hi = nd->hi[k] + pad;
        if (fabs(d[k]) < 1e-300) {
            if (o[k] < lo || o[k] > hi) return 0;
            continue;
        }
        double a = (lo - o[k]) / d[k], b = (hi - o[k]) / d[k];
        if (a > b) { double x = a; a = b; b = x; }
        t0 = fmax(t0, a);
        t1 = fmin(t1, b);
        if (t0 > t1) return 0;
    }
    return 1;
}

/* Any-hit query.  Returns TRI_HIT if some triangle is hit robustly, TRI_MISS
 * if every triangle is missed robustly, TRI_NEAR otherwise.  brute != 0 tests
 * every triangle; otherwise the BVH, with boxes padded by the tolerance at the
 * farthest distance any scene point can be, so it never skips a triangle the
 * brute-force loop would classify as hit or near. */
int orc_anyhit(const orc_scene* s, const double o[3], const double d_in[3], double delta_abs,
               double delta_rel, int brute)
{
    if (s->ntri == 0) return TRI_MISS;
    double dl = norm3(d_in);
    double d[3] = {d_in[0] / dl, d_in[1] / dl, d_in[2] / dl};
    double e1[3], e2[3];
    onb(d, d[2] >= 0.0 ? 1.0 : -1.0, e1, e2);
    int near = 0;
    if (brute) {
        for (int64_t f = 0; f < s->ntri; ++f) {
            int r = classify_tri(s->v + f * 9, o, d, e1, e2, delta_abs, delta_rel);
            if (r == TRI_HIT) return TRI_HIT;
            if (r == TRI_NEAR) near = 1;
        }
        return near ? TRI_NEAR : TRI_MISS;
    }
    double oc[3] = {o[0] - s->center[0], o[1] - s->center[1], o[2] - s->center[2]};
    double tfar = norm3(oc) + 0.5 * s->diag;
    double pad = delta_abs + delta_rel * tfar;
    int32_t stack[256];
    int sp = 0;
    stack[sp++] = 0;
    while (sp > 0) {
        const onode* nd = &s->nodes[stack[--sp]];
        if (!box_hit_padded(nd, o, d, pad)) continue;
        if (nd->left < 0) {
            for (int32_t q = nd->start; q < nd->start + nd->count; ++q) {
                int r = classify_tri(s->v + (size_t)s->order[q] * 9, o, d, e1, e2, delta_abs, delta_rel);
                if (r == TRI_HIT) return TRI_HIT;
                if (r == TRI_NEAR) near = 1;
            }
        } else {
            stack[sp++] = nd->right;
            stack[sp++] = nd->left;
        }
    }
    return near ? TRI_NEAR : TRI_MISS;
}

/* ------------------------------------------------------------------------ */
/* The estimator                                                              */
/* ------------------------------------------------------------------------ */
typedef struct {
    int32_t n_views, height, width, view_base;
    const float *pos, *nrm, *kd, *korm; /* [3][N] planar; korm = (occlusion, roughness, metallic) */
    const uint8_t* mask;                /* [N] */
    const float* eye;                   /* [n_views][3] */
} orc_gbuffer;

typedef struct {
    int32_t spp;
    uint32_t flags;
    uint64_t seed;
    double tau;
    double ray_eps;
    double delta_vis_abs, delta_vis_rel; /* visibility tolerance (world units, x t) */
    double delta_ang;                    /* texel-boundary tolerance, radians of arc */
    double delta_cos;                    /* tolerance on n.v / n.l sign decisions */
    int32_t brute;                       /* all-triangle visibility instead of the BVH */
    /* Direction-error model of the parity protocol, in units of u = 2^-24
     * (all 0: no conditioning is computed).  An FP32 evaluation of a
     * sampling chain moves the sampled direction by at most
     *   light    dir_light u
     *   cosine   dir_cos u
     *   GGX      (dir_ggx0 + dir_ggx1 (1 + (1 - s) A(g)) (1 + A(h)) / |m|) u
     * where A(x) = 1 / (sqrt(x + dir_arg u) + sqrt(x)) is how much the square
     * root amplifies an absolute error of its argument x, g and h are the
     * arguments of the two square roots of the visible-normal warp, s its
     * blend weight and |m| the length of the un-stretched normal (the
     * normalisation divides the error by it). */
    double dir_light, dir_cos, dir_ggx0, dir_ggx1, dir_arg;
} orc_params;

/* flags: technique subsets of the estimator (the sampling ablation of
 * appendix D compares cosine, BSDF and light-probe sampling with MIS) */
#define ORC_LIGHT_OFF 1u  /* no light sample and p_light == 0: BSDF sampling only */
#define ORC_FORCE_COS 2u  /* q = 1: the BSDF technique is pure cosine */
#define ORC_BSDF_OFF 4u   /* no BSDF sample and no BSDF density in P: light sampling only */
#define ORC_FORCE_GGX 8u  /* q = 0 where n.v > 0: the BSDF technique is pure GGX VNDF */
#define ORC_BILINEAR 16u  /* probe radiance by the bilinear reconstruction instead of the nearest texel */

/* decision record flag bits (shared meaning with the HIP debug dump) */
#define DEC_LOBE_COS   (1u << 0)
#define DEC_L_CULL     (1u << 1)
#define DEC_B_CULL     (1u << 2)
#define DEC_L_TRACED   (1u << 3)
#define DEC_B_TRACED   (1u << 4)
#define DEC_L_HIT      (1u << 5)
#define DEC_B_HIT      (1u << 6)
#define DEC_NOV_POS    (1u << 7)
#define DEC_VALID      (1u << 8)
#define DEC_NONE       0xFFFFFFFFu

#define R_MIN_F 0.08f

typedef struct {
    int valid;
    double p[3], n[3], nlen, V[3], NoV;
    int nov_pos;
    double t[3], b[3];
    double kd[3], r, m, alpha, F0[3];
    float qf;
    int r_active; /* roughness above the clamp: d alpha / d r = 2 r */
} pix_setup;

static int setup_pixel(const orc_gbuffer* g, int64_t pix, pix_setup* S, int* nonfinite)
{
    int64_t N = (int64_t)g->n_views * g->height * g->width;
    memset(S, 0, sizeof(*S));
    *nonfinite = 0;
    if (!g->mask[pix]) return 0;
    int v = (int)(pix / ((int64_t)g->height * g->width));
    float raw[12], eyef[3];
    for (int k = 0; k < 3; ++k) {
        raw[k] = g->pos[k * N + pix];
        raw[3 + k] = g->nrm[k * N + pix];
        raw[6 + k] = g->kd[k * N + pix];
        raw[9 + k] = g->korm[k * N + pix];
        eyef[k] = g->eye[v * 3 + k];
    }
    for (int k = 0; k < 12; ++k) if (!isfinite(raw[k])) { *nonfinite = 1; return 0; }
    for (int k = 0; k < 3; ++k) if (!isfinite(eyef[k])) { *nonfinite = 1; return 0; }
    if (raw[3] == 0.0f && raw[4] == 0.0f && raw[5] == 0.0f) return 0;
    double wv[3];
    for (int k = 0; k < 3; ++k) {
        S->p[k] = raw[k];
        wv[k] = (double)eyef[k] - (double)raw[k];
    }
    if (wv[0] == 0.0 && wv[1] == 0.0 && wv[2] == 0.0) return 0;
    double nr[3] = {raw[3], raw[4], raw[5]};
    S->nlen = norm3(nr);
    for (int k = 0; k < 3; ++k) S->n[k] = nr[k] / S->nlen;
    double vl = norm3(wv);
    for (int k = 0; k < 3; ++k) S->V[k] = wv[k] / vl;
    S->NoV = dot3(S->n, S->V);
    S->nov_pos = S->NoV > 0.0;
    onb(S->n, signbit(raw[5]) ? -1.0 : 1.0, S->t, S->b);
    for (int k = 0; k < 3; ++k) S->kd[k] = raw[6 + k];
    S->r = raw[10];
    S->m = raw[11];
    S->r_active = raw[10] > R_MIN_F;
    double rc = S->r_active ? (double)raw[10] : (double)R_MIN_F;
    S->alpha = rc * rc;
    for (int k = 0; k < 3; ++k) S->F0[k] = 0.04 * (1.0 - S->m) + S->kd[k] * S->m;
    S->valid = 1;
    return 1;
}

/* Lobe-selection probability, an FP32 decision on both sides. */
static float lobe_q(const pix_setup* S, float m_f, uint32_t flags)
{
    volatile float one_minus = 1.0f - m_f;
    float q = 0.5f * one_minus;
    if (q < 0.0f) q = 0.0f;
    if (q > 1.0f) q = 1.0f;
    if (!S->nov_pos || (flags & ORC_FORCE_COS)) q = 1.0f;
    else if (flags & ORC_FORCE_GGX) q = 0.0f;
    return q;
}

/* Per-sample terms and per-pixel accumulators.  The outputs of a pixel are
 * sums over its samples of terms; each term is itself a sum of products, and
 * the FP32 error of evaluating it is bounded by a small multiple of u times
 * the sum of the absolute values of those summands (`abs`).  The normal
 * gradient is kept in the pixel's tangent frame (t, b): the gradient with
 * respect to the unnormalised normal lies in the tangent plane. */
enum { T_CD = 0, T_CS = 3, T_GKD = 6, T_GR = 9, T_GM = 10, T_GNT = 11, T_GNB = 12, T_COEF = 13, T_N = 16 };
#define O_N T_COEF /* per-pixel accumulated terms: all but the probe coefficients */

typedef struct {
    double v[T_N]; /* the terms */
    double a[T_N]; /* sums of the absolute values of their summands */
} sample_terms;

typedef struct {
    /* outputs of one pixel, in the term layout above */
    double val[O_N];
    double abs[O_N];  /* sum over samples of the summands' absolute values */
    double cond[O_N]; /* sum over samples of |d term / d direction| times the sample's direction-error bound */
    double lerr[O_N]; /* absolute bound on the FP32 error entering through the radiance lookup itself
                         (bilinear coordinates and tap sums; 0 for the nearest texel) */
    double t[3], b[3], nlen; /* tangent frame and |n_raw| of the evaluation side */
    uint32_t hitbits[64]; /* 2 bits per sample, spp <= 1024 */
    int n_synced, n_flag, n_hard;
} pix_out;

typedef struct {
    int32_t texel;
    double coef[3];
    double absc[3];
    double cond[3]; /* |d coef / d direction| times the direction-error bound */
    int bil;        /* bilinear: the coefficient spreads over the tent taps around (x, y) */
    double x, y;    /* continuous texel coordinates of the sample */
    double dx, dy;  /* bound on the FP32 error of (x, y), in texels */
} env_contrib;

/* The terms of one sample at direction w.  `Ss` drives sampling-side
 * quantities (P, q), `Se` the differentiated integrand (they differ only in
 * the frozen-sample finite-difference hook).  pL is the light technique's
 * density at w, L the radiance.  unit_pdf: P = 1 (the bare integrand). */
static void terms_at(const pix_setup* Ss, const pix_setup* Se, double q, const double w[3], double pL,
                     const double* Lv, int spp, double Hv, int grad, const double* Ud, const double* Us,
                     double bsdf_w, int unit_pdf, sample_terms* T)
{
    memset(T, 0, sizeof(*T));
    double NoL = dot3(Se->n, w);
    double h[3] = {Se->V[0] + w[0], Se->V[1] + w[1], Se->V[2] + w[2]};
    double hl = norm3(h);
    for (int k = 0; k < 3; ++k) h[k] /= hl;
    /* sampling-side density (detached) */
    double NoLs = dot3(Ss->n, w);
    double hs[3] = {Ss->V[0] + w[0], Ss->V[1] + w[1], Ss->V[2] + w[2]};
    double hsl = norm3(hs);
    for (int k = 0; k < 3; ++k) hs[k] /= hsl;
    double nxh[3];
    cross3(Ss->n, hs, nxh);
    double pcos = NoLs > 0.0 ? NoLs / ORC_PI : 0.0;
    double pggx = 0.0;
    if (Ss->nov_pos) {
        double a = Ss->alpha;
        double Ds = orc_ggx_D(dot3(Ss->n, hs), dot3(nxh, nxh), a);
        pggx = Ds / (1.0 + orc_ggx_lambda(Ss->NoV, a)) / (4.0 * Ss->NoV);
    }
    /* balance heuristic over the techniques in use: light (density pL, 0
     * when off) and the BSDF mixture (weight 0 when off) */
    double P = unit_pdf ? 1.0 : pL + bsdf_w * (q * pcos + (1.0 - q) * pggx);
    double K = Hv / (P * (double)spp);
    /* diffuse, demodulated (kd applied outside): (1-m)/pi * NoL * L */
    double kdiff = (1.0 - Se->m) / ORC_PI * NoL * K;
    /* specular: F D G2 / (4 NoV) * L, NoL cancelled; the _a values are the
     * sums of the absolute values of the summands of each difference */
    double S = 0.0, Fw = 0.0, dSdr = 0.0, dSdr_a = 0.0, dSdNoV = 0.0, dSdNoV_a = 0.0, dSdNoL = 0.0,
           dSdNoH = 0.0;
    double F[3] = {0, 0, 0};
    if (Ss->nov_pos) {
        double a = Se->alpha, NoV = Se->NoV, NoH = dot3(Se->n, h), VoH = dot3(Se->V, h);
        cross3(Se->n, h, nxh);
        double s2 = dot3(nxh, nxh);
        double D = orc_ggx_D(NoH, s2, a);
        double LV = orc_ggx_lambda(NoV, a), LL = orc_ggx_lambda(NoL, a);
        double G2 = 1.0 / (1.0 + LV + LL);
        S = D * G2 / (4.0 * NoV);
        double omv = 1.0 - VoH;
        Fw = omv * omv * omv * omv * omv;
        for (int c = 0; c < 3; ++c) F[c] = Se->F0[c] + (1.0 - Se->F0[c]) * Fw;
        if (grad) {
            double B = a * a * NoH * NoH + s2;
            double dDda = D * (2.0 / a - 4.0 * a * NoH * NoH / B);
            double dDda_a = D * (2.0 / a + 4.0 * a * NoH * NoH / B);
            double dlv = lambda_dalpha(NoV, a), dll = lambda_dalpha(NoL, a);
            double dSda = (dDda * G2 - D * G2 * G2 * (dlv + dll)) / (4.0 * NoV);
            double dSda_a = (dDda_a * G2 + D * G2 * G2 * (fabs(dlv) + fabs(dll))) / (4.0 * NoV);
            dSdr = Se->r_active ? dSda * 2.0 * Se->r : 0.0;
            dSdr_a = Se->r_active ? dSda_a * 2.0 * fabs(Se->r) : 0.0;
            double dDdc = D * 4.0 * (1.0 - a * a) * NoH / B;
            double dG2dV = -G2 * G2 * lambda_dx(NoV, a);
            double dG2dL = -G2 * G2 * lambda_dx(NoL, a);
            dSdNoV = D * dG2dV / (4.0 * NoV) - S / NoV;
            dSdNoV_a = fabs(D * dG2dV / (4.0 * NoV)) + fabs(S / NoV);
            dSdNoL = D * dG2dL / (4.0 * NoV);
            dSdNoH = dDdc * G2 / (4.0 * NoV);
        }
    }
    for (int c = 0; c < 3; ++c) {
        const double L = Lv[c];
        T->v[T_CD + c] = kdiff * L;
        T->a[T_CD + c] = fabs(kdiff * L);
        T->v[T_CS + c] = F[c] * S * K * L;
        T->a[T_CS + c] = fabs(F[c] * S * K * L);
    }
    if (!grad) return;
    double gnd = 0.0, gns = 0.0, gnd_a = 0.0, gns_a = 0.0;
    for (int c = 0; c < 3; ++c) {
        const double L = Lv[c];
        const double akd = Us[c] * Se->m * (1.0 - Fw) * S * K;
        const double am1 = Ud[c] * (-NoL / ORC_PI) * K;
        const double am2 = Us[c] * (Se->kd[c] - 0.04) * (1.0 - Fw) * S * K;
        const double am2_a = fabs(Us[c]) * (fabs(Se->kd[c]) + 0.04) * (1.0 - Fw) * S * fabs(K);
        T->v[T_GKD + c] = akd * L;
        T->a[T_GKD + c] = fabs(akd * L);
        T->v[T_GM] += am1 * L + am2 * L;
        T->a[T_GM] += fabs(am1 * L) + am2_a * fabs(L);
        T->v[T_GR] += Us[c] * F[c] * K * dSdr * L;
        T->a[T_GR] += fabs(Us[c] * F[c] * K * L) * dSdr_a;
        gnd += Ud[c] * (1.0 - Se->m) / ORC_PI * L * K;
        gns += Us[c] * F[c] * L * K;
        gnd_a += fabs(Ud[c] * (1.0 - Se->m) / ORC_PI * L * K);
        gns_a += fabs(Us[c] * F[c] * L * K);
        T->v[T_COEF + c] = Ud[c] * kdiff + Us[c] * F[c] * S * K;
        T->a[T_COEF + c] = fabs(Ud[c] * kdiff) + fabs(Us[c] * F[c] * S * K);
    }
    /* d/dn of the sample (the view and half vectors held fixed), in the
     * tangent frame: gnd w + gns (dS/dNoV V + dS/dNoL w + dS/dNoH h) */
    const double* fr[2] = {Se->t, Se->b};
    for (int d = 0; d < 2; ++d) {
        const double wt = dot3(w, fr[d]), vt = dot3(Se->V, fr[d]), ht = dot3(h, fr[d]);
        T->v[T_GNT + d] = gnd * wt + gns * (dSdNoV * vt + dSdNoL * wt + dSdNoH * ht);
        T->a[T_GNT + d] = gnd_a * fabs(wt) +
                          gns_a * (dSdNoV_a * fabs(vt) + fabs(dSdNoL * wt) + fabs(dSdNoH * ht));
    }
}

/* unit vectors e1, e2 orthogonal to the unit vector w and to each other */
static void tangent_pair(const double w[3], double e1[3], double e2[3])
{
    const double a[3] = {1.0, 0.0, 0.0}, b[3] = {0.0, 1.0, 0.0};
    cross3(w, fabs(w[0]) < 0.9 ? a : b, e1);
    const double l = norm3(e1);
    for (int k = 0; k < 3; ++k) e1[k] /= l;
    cross3(w, e1, e2);
}

/* Per-sample evaluation at direction w: accumulates the terms, the sums of
 * their summands' magnitudes, their conditioning in the direction and their
 * lookup error into `out`, and fills the probe-gradient contribution.
 *   pL      the light technique's density at w (0 when off or none)
 *   pl_num  its numerator pdf_uv / (2 pi^2): the density at a nearby direction
 *           w' of the same texel is pl_num / sin(theta(w'))
 *   e_dir   the sample's direction-error bound (radians; 0: no conditioning).
 *           The conditioning of each term is |grad_w term| e_dir, with the
 *           gradient over the directions orthogonal to w taken by central
 *           differences (texel, radiance and visibility held fixed).
 * unit_pdf (the bare integrand): P = 1 and the conditioning is the old
 * one-ulp measure |term| u / |n.l|. */
static void eval_sample(const pix_setup* Ss, const pix_setup* Se, float qf, const double w[3], double pL,
                        double pl_num, const double* Lv, const double* dLv, int spp, double Hv, int grad,
                        const double* Ud, const double* Us, pix_out* out, env_contrib* ec, double bsdf_w,
                        double e_dir, int unit_pdf)
{
    const double q = (double)qf;
    sample_terms T;
    terms_at(Ss, Se, q, w, pL, Lv, spp, Hv, grad, Ud, Us, bsdf_w, unit_pdf, &T);
    double cond[T_N] = {0};
    if (unit_pdf) {
        const double cu = 0x1p-24 / fmax(fabs(dot3(Se->n, w)), 1e-30);
        for (int i = 0; i < T_N; ++i) cond[i] = T.a[i] * cu;
    } else if (e_dir > 0.0) {
        const double eps = 1e-6;
        double e[2][3], g2[T_N] = {0};
        tangent_pair(w, e[0], e[1]);
        for (int d = 0; d < 2; ++d) {
            sample_terms Tp[2];
            for (int sg = 0; sg < 2; ++sg) {
                double wp[3];
                for (int k = 0; k < 3; ++k) wp[k] = w[k] + (sg ? -eps : eps) * e[d][k];
                const double l = norm3(wp);
                for (int k = 0; k < 3; ++k) wp[k] /= l;
                const double rho = sqrt(wp[0] * wp[0] + wp[2] * wp[2]);
                const double pLp = (pl_num > 0.0 && rho > 0.0) ? pl_num / rho : 0.0;
                terms_at(Ss, Se, q, wp, pLp, Lv, spp, Hv, grad, Ud, Us, bsdf_w, unit_pdf, &Tp[sg]);
            }
            for (int i = 0; i < T_N; ++i) {
                const double dd = (Tp[0].v[i] - Tp[1].v[i]) / (2.0 * eps);
                g2[i] += dd * dd;
            }
        }
        for (int i = 0; i < T_N; ++i) cond[i] = sqrt(g2[i]) * e_dir;
    }
    /* the lookup error: every term is linear in the radiance, so its change
     * is bounded by the coefficient of each channel times that channel's
     * radiance bound */
    double lerr[T_N] = {0};
    if (dLv[0] > 0.0 || dLv[1] > 0.0 || dLv[2] > 0.0) {
        for (int c = 0; c < 3; ++c) {
            double unit[3] = {0.0, 0.0, 0.0};
            unit[c] = 1.0;
            sample_terms Tc;
            terms_at(Ss, Se, q, w, pL, unit, spp, Hv, grad, Ud, Us, bsdf_w, unit_pdf, &Tc);
            for (int i = 0; i < T_N; ++i) lerr[i] += fabs(Tc.v[i]) * dLv[c];
        }
    }
    for (int i = 0; i < O_N; ++i) {
        out->val[i] += T.v[i];
        out->abs[i] += T.a[i];
        out->cond[i] += cond[i];
        out->lerr[i] += lerr[i];
    }
    for (int c = 0; c < 3; ++c) {
        ec->coef[c] = T.v[T_COEF + c];
        ec->absc[c] = T.a[T_COEF + c];
        ec->cond[c] = cond[T_COEF + c];
    }
}

typedef struct {
    const orc_scene* scene;
    const orc_env* env_s;     /* sampling tables + radiance */
    const float* env_eval;    /* radiance for the integrand (FD hook) or NULL */
    const orc_gbuffer* gs;    /* sampling G-buffer */
    const orc_gbuffer* ge;    /* evaluation G-buffer (FD hook) or NULL */
    const orc_params* prm;
    const uint32_t* sync;     /* [npix][spp][3] decisions of the HIP path or NULL */
    uint32_t* dec_out;        /* [npix][spp][3] or NULL */
    double* dir_out;          /* [npix][spp][2][4] sampled direction and its error bound, or NULL */
} shade_ctx;

/* Direction-error bound (radians) of a sample drawn by an FP32 evaluation of
 * its sampling chain; the constants are the parity protocol's (orc_params). */
static double dir_err_ggx(const orc_params* P, const vndf_aux* a)
{
    const double u = 0x1p-24, d = P->dir_arg * u;
    const double g = fmax(a->g, 0.0), h = fmax(a->h, 0.0);
    const double Ag = 1.0 / (sqrt(g + d) + sqrt(g));
    const double Ah = 1.0 / (sqrt(h + d) + sqrt(h));
    return u * (P->dir_ggx0 + P->dir_ggx1 * (1.0 + (1.0 - a->s) * Ag) * (1.0 + Ah) / fmax(a->mlen, 1e-300));
}

static void shade_pixel(const shade_ctx* C, int64_t q, int64_t pix, int grad, const double* Ud,
                        const double* Us, pix_out* out, env_contrib* ecs, int64_t* nonfinite)
{
    const orc_params* P = C->prm;
    const orc_env* E = C->env_s;
    const float* envL = C->env_eval ? C->env_eval : E->env;
    int spp = P->spp;
    const double u = 0x1p-24;
    const int want_cond = P->dir_light > 0.0 || P->dir_cos > 0.0 || P->dir_ggx0 > 0.0 || P->dir_ggx1 > 0.0;
    memset(out, 0, sizeof(*out));
    for (int s = 0; s < 2 * spp; ++s) ecs[s].texel = -1;
    pix_setup Ss, Se;
    int nf = 0;
    int ok = setup_pixel(C->gs, pix, &Ss, &nf);
    if (nf) (*nonfinite)++;
    const uint32_t* sy = C->sync ? C->sync + (size_t)q * spp * 3 : NULL;
    uint32_t* dq = C->dec_out ? C->dec_out + (size_t)q * spp * 3 : NULL;
    double* dirq = C->dir_out ? C->dir_out + (size_t)q * spp * 8 : NULL;
    if (dirq) for (int k = 0; k < 8 * spp; ++k) dirq[k] = NAN;
    if (!ok) {
        if (dq) for (int s = 0; s < spp; ++s) { dq[s * 3] = DEC_NONE; dq[s * 3 + 1] = DEC_NONE; dq[s * 3 + 2] = 0; }
        if (sy && (sy[2] & DEC_VALID)) out->n_hard++;
        return;
    }
    if (sy && !(sy[2] & DEC_VALID)) out->n_hard++;
    /* n.v sign: synced when within tolerance */
    if (fabs(Ss.NoV) < P->delta_cos && sy) {
        int g = (sy[2] & DEC_NOV_POS) != 0;
        if (g != Ss.nov_pos) { Ss.nov_pos = g; }
        out->n_synced++;
    } else if (sy && (((sy[2] & DEC_NOV_POS) != 0) != Ss.nov_pos)) {
        out->n_hard++;
    }
    if (C->ge) {
        int nf2 = 0;
        if (!setup_pixel(C->ge, pix, &Se, &nf2)) Se = Ss;
        Se.nov_pos = Ss.nov_pos;
    } else {
        Se = Ss;
    }
    float m_f = C->gs->korm[2 * ((int64_t)C->gs->n_views * C->gs->height * C->gs->width) + pix];
    float qf = lobe_q(&Ss, m_f, P->flags);
    int light_on = E->light_enabled && !(P->flags & ORC_LIGHT_OFF);
    int bsdf_on = !(P->flags & ORC_BSDF_OFF);
    int64_t HW = (int64_t)C->gs->height * C->gs->width;
    uint32_t view = (uint32_t)(pix / HW), piv = (uint32_t)(pix % HW);
    double origin[3];
    for (int k = 0; k < 3; ++k) origin[k] = Ss.p[k] + P->ray_eps * Ss.n[k];
    double Vl[3] = {dot3(Ss.V, Ss.t), dot3(Ss.V, Ss.b), Ss.NoV};
    const double two_pi2 = 2.0 * ORC_PI * ORC_PI;
    for (int s = 0; s < spp; ++s) {
        double xi[8];
        sample_uniforms(P->seed, piv, (uint32_t)C->gs->view_base + view, (uint32_t)s, xi);
        uint32_t rec0 = DEC_NONE, rec1 = DEC_NONE, rec2 = DEC_VALID | (Ss.nov_pos ? DEC_NOV_POS : 0u);
        const uint32_t* gsr = sy ? sy + s * 3 : NULL;
        for (int tech = 0; tech < 2; ++tech) {
            double w[3], pL = 0.0, pl_num = 0.0;
            double e_dir = 0.0;   /* bound on the FP32 direction's distance from w (radians) */
            int ti = -1, tj = -1;
            double tex_margin = INFINITY;
            double bx = 0.0, by = 0.0, bdx = 0.0, bdy = 0.0; /* texel coordinates and error bounds */
            if (tech == 0) {
                if (!light_on) continue;
                int32_t a, b;
                sample_light_xy(E, xi[0], xi[1], w, &pL, &a, &b, &bx, &by);
                ti = a; tj = b;
                pl_num = (double)E->pdf[(size_t)ti * E->W + tj] / two_pi2;
                e_dir = P->dir_light * u;
                /* FP32: one quotient of table differences plus the integer part */
                bdx = 2.0 * u * (bx + 8.0);
                bdy = 2.0 * u * (by + 8.0);
                rec0 = (uint32_t)(ti * E->W + tj);
                if (gsr && gsr[0] != rec0) out->n_hard++;
                if (!(pL > 0.0)) { rec2 |= DEC_L_CULL; continue; }
            } else {
                if (!bsdf_on) continue;
                double loc[3];
                int cosl = (float)xi[2] < qf;
                if (cosl) {
                    rec2 |= DEC_LOBE_COS;
                    orc_sample_cos_local(xi[4], xi[5], loc);
                    e_dir = P->dir_cos * u;
                } else {
                    vndf_aux aux;
                    double lensq = sample_vndf_aux(Vl, Ss.alpha, xi[4], xi[5], loc, &aux);
                    if (lensq < 1e-14) out->n_flag++;
                    e_dir = want_cond ? dir_err_ggx(P, &aux) : 0.0;
                }
                if (gsr && (((gsr[2] & DEC_LOBE_COS) != 0) != cosl)) out->n_hard++;
                for (int k = 0; k < 3; ++k) w[k] = loc[0] * Ss.t[k] + loc[1] * Ss.b[k] + loc[2] * Ss.n[k];
                double wl = norm3(w);
                for (int k = 0; k < 3; ++k) w[k] /= wl;
                texel_of_dir_xy(E->H, E->W, w, &ti, &tj, &tex_margin, &bx, &by);
                {
                    /* FP32 error of the coordinates: the direction error
                     * (twice its bound; 64 u without a direction model)
                     * through theta and phi = atan2, plus the roundoff of
                     * atan2 and of the scaling */
                    const double dw = e_dir > 0.0 ? 2.0 * e_dir : 64.0 * u;
                    const double rho = sqrt(w[0] * w[0] + w[2] * w[2]);
                    bdy = (dw + 8.0 * u * ORC_PI) * (double)E->H / ORC_PI + 4.0 * u * by;
                    bdx = (rho > 0.0 ? dw / rho : (double)E->W) * (double)E->W / (2.0 * ORC_PI) +
                          16.0 * u * ORC_PI * (double)E->W / (2.0 * ORC_PI) + 4.0 * u * bx;
                    bdx = fmin(bdx, (double)E->W);
                    bdy = fmin(bdy, (double)E->H);
                }
                uint32_t mine = (uint32_t)(ti * E->W + tj);
                if (gsr && gsr[1] != DEC_NONE && gsr[1] != mine) {
                    /* undecided in FP32 within the tolerance or within twice
                     * the sample's own direction-error bound */
                    if (tex_margin < fmax(P->delta_ang, 2.0 * e_dir)) {
                        ti = (int)(gsr[1] / (uint32_t)E->W);
                        tj = (int)(gsr[1] % (uint32_t)E->W);
                        out->n_synced++;
                    } else {
                        out->n_hard++;
                    }
                }
                rec1 = (uint32_t)(ti * E->W + tj);
                if (light_on) {
                    double rho = sqrt(w[0] * w[0] + w[2] * w[2]);
                    pl_num = (double)E->pdf[(size_t)ti * E->W + tj] / two_pi2;
                    pL = rho > 0.0 ? pl_num / rho : 0.0;
                }
            }
            if (dirq) {
                for (int k = 0; k < 3; ++k) dirq[(s * 2 + tech) * 4 + k] = w[k];
                dirq[(s * 2 + tech) * 4 + 3] = e_dir;
            }
            uint32_t bit_cull = tech ? DEC_B_CULL : DEC_L_CULL;
            uint32_t bit_tr = tech ? DEC_B_TRACED : DEC_L_TRACED;
            uint32_t bit_hit = tech ? DEC_B_HIT : DEC_L_HIT;
            double NoL = dot3(Ss.n, w);
            int cull = !(NoL > 0.0);
            if (gsr && fabs(NoL) < fmax(P->delta_cos, 2.0 * e_dir)) {
                int gc = (gsr[2] & bit_cull) != 0;
                if (gc != cull) { cull = gc; out->n_synced++; }
            } else if (gsr && (((gsr[2] & bit_cull) != 0) != cull)) {
                out->n_hard++;
            }
            if (cull) { rec2 |= bit_cull; continue; }
            double Hv = 1.0;
            if (P->tau != 0.0) {
                rec2 |= bit_tr;
                int r = orc_anyhit(C->scene, origin, w, P->delta_vis_abs, P->delta_vis_rel, P->brute);
                int hit;
                if (r == TRI_NEAR) {
                    if (gsr) { hit = (gsr[2] & bit_hit) != 0; out->n_synced++; }
                    else { hit = 1; out->n_flag++; }
                } else {
                    hit = r == TRI_HIT;
                    if (gsr && (((gsr[2] & bit_hit) != 0) != hit)) out->n_hard++;
                }
                if (hit) {
                    rec2 |= bit_hit;
                    int bitpos = 2 * s + tech;
                    out->hitbits[bitpos >> 5] |= 1u << (bitpos & 31);
                    Hv = 1.0 - P->tau;
                }
            }
            if (Hv == 0.0) continue;   /* no incident radiance (appendix A) */
            double Lv[3], dLv[3] = {0.0, 0.0, 0.0};
            const int bil = (P->flags & ORC_BILINEAR) != 0;
            if (bil) {
                orc_probe_bilinear(envL, E->H, E->W, bx, by, Lv);
                bilinear_shift_bound(envL, E->H, E->W, bx, by, bdx, bdy, dLv);
            } else {
                const float* Lrad = envL + ((size_t)ti * E->W + tj) * 3;
                for (int c = 0; c < 3; ++c) Lv[c] = (double)Lrad[c];
            }
            env_contrib* ec = &ecs[2 * s + tech];
            eval_sample(&Ss, &Se, qf, w, pL, light_on ? pl_num : 0.0, Lv, dLv, spp, Hv, grad, Ud, Us, out, ec,
                        bsdf_on ? 1.0 : 0.0, e_dir, 0);
            ec->texel = ti * E->W + tj;
            ec->bil = bil;
            ec->x = bx;
            ec->y = by;
            ec->dx = bdx;
            ec->dy = bdy;
        }
        if (dq) { dq[s * 3] = rec0; dq[s * 3 + 1] = rec1; dq[s * 3 + 2] = rec2; }
    }
    for (int k = 0; k < 3; ++k) {
        out->t[k] = Se.t[k];
        out->b[k] = Se.b[k];
    }
    out->nlen = Se.nlen;
}

/* Probe gradient of one bilinear sample: the coefficient of the radiance
 * times each tap's tent weight.  The lookup error (lenv) adds, for every tap
 * an FP32 error of (dx, dy) in the coordinates can reach, the coefficient
 * times the bound on its weight's change (tent weights are 1-Lipschitz). */
static void scatter_bilinear(const env_contrib* e, int H, int W, double* genv, double* senv, double* cenv,
                             double* lenv)
{
    const double xs = e->x - 0.5, ys = e->y - 0.5;
    const double ex = fmin(e->dx, 1.0), ey = fmin(e->dy, 1.0);
    const int ja = (int)floor(xs - e->dx), jb = (int)floor(xs + e->dx) + 1;
    const int ia = (int)floor(ys - e->dy), ib = (int)floor(ys + e->dy) + 1;
    for (int i = ia; i <= ib; ++i)
        for (int j = ja; j <= jb; ++j) {
            const double tx = tent(xs, j), ty = tent(ys, i);
            const double wt = tx * ty;
            const double werr = ex * fmin(ty + ey, 1.0) + tx * ey;
            const size_t t = (size_t)clamp_row(i, H) * W + wrap_col(j, W);
            for (int c = 0; c < 3; ++c) {
                genv[t * 3 + c] += e->coef[c] * wt;
                if (senv) senv[t * 3 + c] += e->absc[c] * wt;
                if (cenv) cenv[t * 3 + c] += e->cond[c] * wt;
                if (lenv) lenv[t * 3 + c] += e->absc[c] * werr;
            }
        }
}

/* Forward (grad == 0) or backward (grad == 1) over a list of pixels.
 * Outputs are [3][npix] in list order.  info = [npix][3]: synced decisions,
 * unsyncable (flagged) decisions, hard mismatches against `sync`.
 * vaux (or NULL) = [3][15][npix]: for each of the 15 per-pixel outputs (c_d,
 * c_s, g_kd, g_korm, g_nrm; 3 channels each) the sum of the absolute values
 * of the summands of its terms, the conditioning of its terms in their
 * sampled directions, and the bound on the error that enters through the
 * radiance lookup.  dir_out (or NULL) = [npix][spp][2][4]: each sample's
 * direction (light, then BSDF technique) and its direction-error bound; NaN
 * where no direction was drawn. */
int64_t orc_shade(const orc_scene* scene, const orc_env* env_s, const float* env_eval,
                  const orc_gbuffer* gs, const orc_gbuffer* ge, const int64_t* pix, int64_t npix,
                  const orc_params* prm, const uint32_t* sync, int grad, const double* Ud,
                  const double* Us, double* cd, double* cs, double* vaux, double* gkd, double* gkorm,
                  double* gn,
                  double* genv, double* senv, double* cenv, double* lenv, uint32_t* hitbits, int32_t hit_words,
                  uint32_t* dec_out, double* dir_out, int32_t* info, int nthreads)
{
    shade_ctx C = {scene, env_s, env_eval, gs, ge, prm, sync, dec_out, dir_out};
    int spp = prm->spp;
    if (spp < 1 || spp > 1024 || hit_words > 64) return -1;
    /* pixels are taken in chunks, and the probe-gradient contributions of a
     * chunk are added in list order after it: the same fixed order as one
     * pass, with bounded memory */
    const int64_t chunk = 65536;
    env_contrib* all = NULL;
    if (grad && genv) all = (env_contrib*)malloc(sizeof(env_contrib) * (size_t)(npix < chunk ? npix : chunk) * 2 * spp);
    int64_t nonfinite = 0;
    int nt = 1;  // a thread count for this call only (num_threads clause)
#ifdef _OPENMP
    nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
    (void)nt;
    for (int64_t q0 = 0; q0 < npix; q0 += chunk) {
        const int64_t q1 = npix - q0 < chunk ? npix : q0 + chunk;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : nonfinite) num_threads(nt)
        for (int64_t q = q0; q < q1; ++q) {
            pix_out o;
            env_contrib local[2 * 256];
            // above 256 samples the pixel's records go to the heap (worker
            // threads may have small stacks)
            env_contrib* big = (!all && spp > 256) ? (env_contrib*)malloc(sizeof(env_contrib) * 2 * (size_t)spp) : NULL;
            env_contrib* ec = all ? all + (size_t)(q - q0) * 2 * spp : (big ? big : local);
            double ud[3] = {0, 0, 0}, us[3] = {0, 0, 0};
            if (grad) for (int c = 0; c < 3; ++c) { ud[c] = Ud[c * npix + q]; us[c] = Us[c * npix + q]; }
            shade_pixel(&C, q, pix[q], grad, ud, us, &o, ec, &nonfinite);
            const double il = o.nlen > 0.0 ? 1.0 / o.nlen : 0.0;
            for (int c = 0; c < 3; ++c) {
                if (cd) cd[c * npix + q] = o.val[T_CD + c];
                if (cs) cs[c * npix + q] = o.val[T_CS + c];
                if (grad) {
                    if (gkd) gkd[c * npix + q] = o.val[T_GKD + c];
                    /* d/dn_raw = (I - n n^T) d/dn / |n_raw| = (t (t.g) + b (b.g)) / |n_raw| */
                    if (gn) gn[c * npix + q] = (o.val[T_GNT] * o.t[c] + o.val[T_GNB] * o.b[c]) * il;
                }
            }
            if (grad && gkorm) {
                gkorm[0 * npix + q] = 0.0;
                gkorm[1 * npix + q] = o.val[T_GR];
                gkorm[2 * npix + q] = o.val[T_GM];
            }
            if (vaux) {
                const double* src[3] = {o.abs, o.cond, o.lerr};
                for (int kind = 0; kind < 3; ++kind) {
                    const double* x = src[kind];
                    double* dst = vaux + (size_t)kind * 15 * npix;
                    for (int c = 0; c < 3; ++c) {
                        dst[(0 + c) * npix + q] = x[T_CD + c];
                        dst[(3 + c) * npix + q] = x[T_CS + c];
                        dst[(6 + c) * npix + q] = x[T_GKD + c];
                        dst[(9 + c) * npix + q] = c == 0 ? 0.0 : (c == 1 ? x[T_GR] : x[T_GM]);
                        dst[(12 + c) * npix + q] = (x[T_GNT] * fabs(o.t[c]) + x[T_GNB] * fabs(o.b[c])) * il;
                    }
                }
            }
            if (hitbits) for (int k = 0; k < hit_words; ++k) hitbits[(size_t)q * hit_words + k] = o.hitbits[k];
            if (info) { info[q * 3] = o.n_synced; info[q * 3 + 1] = o.n_flag; info[q * 3 + 2] = o.n_hard; }
            free(big);
        }
        if (all) {
            /* fixed order: pixel list order, then sample, then technique */
            for (int64_t k = 0; k < (q1 - q0) * 2 * spp; ++k) {
                if (all[k].texel < 0) continue;
                if (all[k].bil) {
                    scatter_bilinear(&all[k], env_s->H, env_s->W, genv, senv, cenv, lenv);
                    continue;
                }
                for (int c = 0; c < 3; ++c) {
                    genv[(size_t)all[k].texel * 3 + c] += all[k].coef[c];
                    if (senv) senv[(size_t)all[k].texel * 3 + c] += all[k].absc[c];
                    if (cenv) cenv[(size_t)all[k].texel * 3 + c] += all[k].cond[c];
                }
            }
        }
    }
    free(all);
    return nonfinite;
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------------ */
/* Batched entry points used by the pin tests (plain loops).                 */
/* ------------------------------------------------------------------------ */
void orc_batch_philox(int64_t n, const uint32_t* ctr, const uint32_t key[2], uint32_t* out)
{
    for (int64_t i = 0; i < n; ++i) orc_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

void orc_batch_uniforms(int64_t n, uint64_t seed, const uint32_t* pix, const uint32_t* view,
                        const uint32_t* s, double* xi)
{
    for (int64_t i = 0; i < n; ++i) sample_uniforms(seed, pix[i], view[i], s[i], xi + 8 * i);
}

void orc_batch_sample_light(const orc_env* e, int64_t n, const double* xi0, const double* xi1,
                            double* w, double* p, int32_t* ti, int32_t* tj, double* x, double* y)
{
    for (int64_t i = 0; i < n; ++i) {
        double a, b;
        sample_light_xy(e, xi0[i], xi1[i], w + 3 * i, p + i, ti + i, tj + i, &a, &b);
        if (x) x[i] = a;
        if (y) y[i] = b;
    }
}

void orc_batch_pdf_light(const orc_env* e, int64_t n, const double* w, double* p)
{
    for (int64_t i = 0; i < n; ++i) p[i] = orc_pdf_light(e, w + 3 * i);
}

void orc_batch_texel_of_dir(int H, int W, int64_t n, const double* w, int32_t* ti, int32_t* tj,
                            double* margin, double* x, double* y)
{
    for (int64_t i = 0; i < n; ++i) {
        int a, b;
        texel_of_dir_xy(H, W, w + 3 * i, &a, &b, margin + i, x ? x + i : NULL, y ? y + i : NULL);
        ti[i] = a;
        tj[i] = b;
    }
}

void orc_batch_probe_bilinear(const float* env, int H, int W, int64_t n, const double* x, const double* y,
                              double* L)
{
    for (int64_t i = 0; i < n; ++i) orc_probe_bilinear(env, H, W, x[i], y[i], L + 3 * i);
}

void orc_batch_pdf_ggx_local(int64_t n, const double* V, double alpha, const double* L, double* p)
{
    for (int64_t i = 0; i < n; ++i) p[i] = orc_pdf_ggx_local(V, L + 3 * i, alpha);
}

void orc_batch_pdf_cos_local(int64_t n, const double* L, double* p)
{
    for (int64_t i = 0; i < n; ++i) p[i] = orc_pdf_cos_local(L + 3 * i);
}

void orc_batch_sample_vndf_local(int64_t n, const double* V, double alpha, const double* u1,
                                 const double* u2, double* L)
{
    for (int64_t i = 0; i < n; ++i) orc_sample_vndf_local(V, alpha, u1[i], u2[i], L + 3 * i);
}

void orc_batch_sample_cos_local(int64_t n, const double* u1, const double* u2, double* L)
{
    for (int64_t i = 0; i < n; ++i) orc_sample_cos_local(u1[i], u2[i], L + 3 * i);
}

void orc_batch_ggx(int64_t n, const double* noh, const double* s2, const double* nov,
                   double alpha, double* D, double* lambda)
{
    for (int64_t i = 0; i < n; ++i) {
        D[i] = orc_ggx_D(noh[i], s2[i], alpha);
        lambda[i] = orc_ggx_lambda(nov[i], alpha);
    }
}

void orc_batch_anyhit(const orc_scene* s, int64_t n, const double* o, const double* d,
                      double delta_abs, double delta_rel, int brute, int32_t* out)
{
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) out[i] = orc_anyhit(s, o + 3 * i, d + 3 * i, delta_abs, delta_rel, brute);
}

/* The integrand of the direct-illumination integral of one pixel at unit
 * directions w: g_d = (1-m)/pi (n.w) L(w) H(w) and g_s = F D G2/(4 n.v) L(w)
 * H(w), zero below the horizon, nearest-texel radiance (bilinear with
 * ORC_BILINEAR in the flags), all-triangle visibility (an undecided ray counts
 * as hit).  Used by the quadrature pins. */
void orc_integrand(const orc_scene* scene, const orc_env* E, const orc_gbuffer* g, int64_t pix,
                   const orc_params* P, int64_t n, const double* w, double* gd, double* gs)
{
    pix_setup S;
    int nf = 0;
    if (!setup_pixel(g, pix, &S, &nf)) {
        memset(gd, 0, sizeof(double) * 3 * (size_t)n);
        memset(gs, 0, sizeof(double) * 3 * (size_t)n);
        return;
    }
    double origin[3];
    for (int k = 0; k < 3; ++k) origin[k] = S.p[k] + P->ray_eps * S.n[k];
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < n; ++i) {
        const double* wi = w + 3 * i;
        pix_out o;
        env_contrib ec;
        memset(&o, 0, sizeof(o));
        if (dot3(S.n, wi) > 0.0) {
            double Hv = 1.0;
            if (P->tau != 0.0 && orc_anyhit(scene, origin, wi, 0.0, 0.0, P->brute) != TRI_MISS)
                Hv = 1.0 - P->tau;
            int ti, tj;
            double m, x, y, Lv[3], dLv[3] = {0.0, 0.0, 0.0};
            texel_of_dir_xy(E->H, E->W, wi, &ti, &tj, &m, &x, &y);
            if (P->flags & ORC_BILINEAR) {
                orc_probe_bilinear(E->env, E->H, E->W, x, y, Lv);
            } else {
                const float* Lrad = E->env + ((size_t)ti * E->W + tj) * 3;
                for (int c = 0; c < 3; ++c) Lv[c] = (double)Lrad[c];
            }
            if (Hv != 0.0)   /* a blocked direction carries no radiance with H = 0 */
                eval_sample(&S, &S, 1.0f, wi, 0.0, 0.0, Lv, dLv, 1, Hv, 0, NULL, NULL, &o, &ec, 1.0, 0.0, 1);
        }
        for (int c = 0; c < 3; ++c) {
            gd[3 * i + c] = o.val[T_CD + c];
            gs[3 * i + c] = o.val[T_CS + c];
        }
    }
}

/* ------------------------------------------------------------------------ */
/* Visibility gradients of the shadow term by edge sampling.  The estimator  */
/* above detaches visibility (section 3.1, "Shadow gradients"); the paper's  */
/* ablation on shadow gradients (appendix "Visibility Gradients from        */
/* Shadows") adds the derivative of the shadowed hemisphere integral with   */
/* respect to the occluding geometry.  Here that derivative is estimated by */
/* sampling mesh edges (the boundary-integral form of the derivative of an  */
/* integral over a moving region).                                           */
/*                                                                           */
/* Seen from the shadow-ray origin o, the region of directions blocked by a */
/* triangle is bounded by the great-circle arcs of its edges.  For an edge  */
/* a-b, a point x(t) = a + t (b - a), t in [0, 1), has direction            */
/* w = (x - o)/r, r = |x - o|.  The arc lies in the plane through o with    */
/* normal m = (a - o) x (b - o), and as the vertices move the arc moves     */
/* along mh = m/|m| at the rate mh . ((1-t) da + t db) / r.  The arc length */
/* per unit t is |(b - a) x w| / r.  When the integrand jumps across the    */
/* arc from h_in (the side of the edge's own face) to h_out, the            */
/* derivative of the integral is the integral along the arc of             */
/* s (h_out - h_in) (mh . dx/dtheta) / r, with s = +1 when the face lies on */
/* the +mh side (the arc moving along +mh uncovers directions) and -1      */
/* otherwise.  With H = 1 - tau on blocked directions, h_in = g (1 - tau)  */
/* (the face blocks) and h_out = g (1 - tau [the out-side ray is blocked]),*/
/* so h_out - h_in = tau g when the out-side ray misses and 0 when          */
/* something else still blocks it.                                           */
/*                                                                           */
/* Only unique edges count, and only silhouettes: an edge whose two faces   */
/* lie on opposite sides of the arc is covered on both sides.  One sample   */
/* draws an edge e with probability p_e (the two-class distribution below) */
/* and t uniformly, so the estimate of d(loss)/d(vertex) adds              */
/*   s tau g(w) |(b - a) x w| / (r^2 p_e n_es) x ((1-t) mh at a, t mh at b) */
/* when the out-side ray misses, where g(w) = sum_c Ud_c g_d,c(w) +         */
/* Us_c g_s,c(w) contracts the integrand of c_d and c_s with the upstream   */
/* gradients.  The out-side ray leaves o along w turned by ORC_EDGE_DELTA   */
/* radians away from the face, normalised.                                  */
/*                                                                           */
/* Random numbers: Philox block 2 of counter (pixel in view, view id, j),   */
/* j the edge sample, gives x0..x3: x2 picks the class, (x0 * n_class) >>   */
/* 32 the edge within it (integers, exact), the 24-bit uniform of x1 is t.  */
/* ------------------------------------------------------------------------ */
#define ORC_EDGE_DELTA (1.0 / 8192.0)

/* Edge classes of the sampling distribution.  An edge is sharp when it has
 * one face, or when the normals of its faces, (b-a)x(c-a) and (a-b)x(d-b),
 * are more than 20 degrees apart: dot < 0, or dot^2 < cos^2(20 deg) |n1|^2
 * |n2|^2.  The test is evaluated in FP32, operation by operation in this
 * order, so that the kernel takes the same decision (it is an integer the
 * sampling depends on).  Sharp edges are K = sharp_gain times as likely per
 * edge as the others: a sample picks the sharp class when (x2 >> 8) (K nS +
 * nR) < K nS 2^24 (exact integers), then an edge uniformly in its class, and
 * weighs it by the class size over the class probability.  The expectation
 * does not depend on K; with K > 1 silhouettes of coarse objects are drawn
 * far more often than under the uniform choice (K = 1). */
#define ORC_SHARP_COS2 0.883022221559489f /* cos^2(20 degrees) */

static int edge_is_sharp(const float* verts, const int32_t* ed)
{
    if (ed[3] < 0) return 1;
    const float* A = verts + 3 * (size_t)ed[0];
    const float* B = verts + 3 * (size_t)ed[1];
    const float* Cc = verts + 3 * (size_t)ed[2];
    const float* D = verts + 3 * (size_t)ed[3];
    float e1[3], e2[3], f1[3], f2[3];
    for (int k = 0; k < 3; ++k) {
        e1[k] = B[k] - A[k];
        e2[k] = Cc[k] - A[k];
        f1[k] = A[k] - B[k];
        f2[k] = D[k] - B[k];
    }
    float n1[3], n2[3];
    n1[0] = e1[1] * e2[2] - e1[2] * e2[1];
    n1[1] = e1[2] * e2[0] - e1[0] * e2[2];
    n1[2] = e1[0] * e2[1] - e1[1] * e2[0];
    n2[0] = f1[1] * f2[2] - f1[2] * f2[1];
    n2[1] = f1[2] * f2[0] - f1[0] * f2[2];
    n2[2] = f1[0] * f2[1] - f1[1] * f2[0];
    float dt = n1[0] * n2[0] + n1[1] * n2[1] + n1[2] * n2[2];
    float q1 = n1[0] * n1[0] + n1[1] * n1[1] + n1[2] * n1[2];
    float q2 = n2[0] * n2[0] + n2[1] * n2[1] + n2[2] * n2[2];
    float lhs = dt * dt;
    float rhs = ORC_SHARP_COS2 * (q1 * q2);
    return dt < 0.0f || lhs < rhs;
}

/* largest radiance per channel over the 3x3 texels around (i, j): bounds the
 * lookup when the nearest texel is undecided */
static void texel_max3(const float* env, int H, int W, int i, int j, double L[3])
{
    for (int c = 0; c < 3; ++c) L[c] = 0.0;
    for (int di = -1; di <= 1; ++di)
        for (int dj = -1; dj <= 1; ++dj) {
            const float* e = texel_ptr(env, H, W, i + di, j + dj);
            for (int c = 0; c < 3; ++c) L[c] = fmax(L[c], fabs((double)e[c]));
        }
}

/* Edge-sampled visibility gradient of the listed pixels, accumulated into
 * gv[n_verts][3].  gv_abs sums |term| per element; gv_cond sums |term|
 * times the FP32 condition of the term (per unit roundoff); gv_flag sums a
 * bound on the terms of samples with an undecided discrete step (silhouette
 * sign, horizon, nearest texel, out-side ray).  counts = {samples, silhouette
 * samples above the horizon, rays traced, rays blocked, flagged samples}.
 * Returns 0, or -1 on bad arguments. */
int orc_edge_grad(const orc_scene* scene, const orc_env* E, const orc_gbuffer* g, const int64_t* pix,
                  int64_t npix, const orc_params* P, int32_t n_es, const int32_t* edges, int64_t n_edges,
                  const float* verts, int64_t n_verts, const double* Ud, const double* Us, double* gv,
                  double* gv_abs, double* gv_cond, double* gv_flag, int64_t* counts, int nthreads,
                  uint32_t sharp_gain)
{
    if (n_es < 0 || n_edges < 0 || n_edges > 0xFFFFFFFFll) return -1;
    for (int k = 0; k < 5; ++k) counts[k] = 0;
    if (n_es == 0 || n_edges == 0 || P->tau == 0.0) return 0;
    const double u = 0x1p-24;
    /* the two classes, each in edge order */
    int64_t* cls = (int64_t*)malloc(sizeof(int64_t) * (size_t)n_edges);
    int64_t nS = 0;
    for (int64_t e = 0; e < n_edges; ++e)
        if (edge_is_sharp(verts, edges + 4 * e)) cls[nS++] = e;
    const int64_t nR = n_edges - nS;
    for (int64_t e = 0, k = nS; e < n_edges; ++e)
        if (!edge_is_sharp(verts, edges + 4 * e)) cls[k++] = e;
    /* sharp_gain: the per-edge weight of the sharp class (1: a uniform choice) */
    const uint64_t gain = sharp_gain ? sharp_gain : 1u;
    const uint64_t Nn = gain * (uint64_t)nS, Dd = Nn + (uint64_t)nR;
    const uint64_t cS = (Nn << 24) / Dd + (((Nn << 24) % Dd) != 0); /* u24 values that pick the sharp class */
    const double wS = cS > 0 ? (double)nS * 16777216.0 / (double)cS : 0.0;
    const double wR = cS < 16777216u ? (double)nR * 16777216.0 / (double)(16777216u - cS) : 0.0;
    int nt = 1;  // a thread count for this call only (num_threads clause)
#ifdef _OPENMP
    nt = nthreads > 0 ? nthreads : omp_get_max_threads();
#endif
    const size_t nv3 = (size_t)n_verts * 3;
    double* acc = (double*)calloc((size_t)nt * 4 * nv3, sizeof(double));
    int64_t* cnt = (int64_t*)calloc((size_t)nt * 5, sizeof(int64_t));
    const int64_t HW = (int64_t)g->height * g->width;
    const uint32_t key[2] = {(uint32_t)P->seed, (uint32_t)(P->seed >> 32)};
#pragma omp parallel num_threads(nt)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double* a_v = acc + (size_t)tid * 4 * nv3;
        double* a_abs = a_v + nv3;
        double* a_cond = a_abs + nv3;
        double* a_flag = a_cond + nv3;
        int64_t* c5 = cnt + (size_t)tid * 5;
#pragma omp for schedule(static)
        for (int64_t q = 0; q < npix; ++q) {
            pix_setup S;
            int nf = 0;
            if (!setup_pixel(g, pix[q], &S, &nf)) continue;
            const double ud[3] = {Ud[q], Ud[npix + q], Ud[2 * npix + q]};
            const double us[3] = {Us[q], Us[npix + q], Us[2 * npix + q]};
            const int nov_near = fabs(S.NoV) < 1e-12;
            double o[3];
            for (int k = 0; k < 3; ++k) o[k] = S.p[k] + P->ray_eps * S.n[k];
            const double olen = norm3(o);
            const uint32_t view = (uint32_t)(pix[q] / HW), piv = (uint32_t)(pix[q] % HW);
            for (int j = 0; j < n_es; ++j) {
                uint32_t ctr[4] = {piv, (uint32_t)g->view_base + view, (uint32_t)j, 2u}, r[4];
                orc_philox4x32_10(ctr, key, r);
                c5[0]++;
                const int sharp = (uint64_t)(r[2] >> 8) * Dd < (Nn << 24);
                const int64_t ncls = sharp ? nS : nR;
                const int64_t e = cls[(sharp ? 0 : nS) + (int64_t)(((uint64_t)r[0] * (uint64_t)ncls) >> 32)];
                const double wcls = sharp ? wS : wR;
                const double t = u01(r[1]);
                const int32_t* ed = edges + 4 * e;
                /* the face sides come from the determinant det(a - o, b - o,
                 * c - o) written with edge vectors, (a - o) . ((b - a) x
                 * (c - a)): the same number, without the cancellation of
                 * differences from a distant o */
                double A[3], qa[3], eab[3], eac[3], ead[3] = {0, 0, 0};
                for (int k = 0; k < 3; ++k) {
                    A[k] = (double)verts[3 * (size_t)ed[0] + k];
                    qa[k] = A[k] - o[k];
                    eab[k] = (double)verts[3 * (size_t)ed[1] + k] - A[k];
                    eac[k] = (double)verts[3 * (size_t)ed[2] + k] - A[k];
                    if (ed[3] >= 0) ead[k] = (double)verts[3 * (size_t)ed[3] + k] - A[k];
                }
                /* a non-finite corner: the sample adds nothing (no decision
                 * the FP32 path takes on it can pass) */
                int finite = 1;
                for (int k = 0; k < 3; ++k)
                    finite &= isfinite(qa[k]) && isfinite(eab[k]) && isfinite(eac[k]) && isfinite(ead[k]);
                if (!finite) continue;
                double m[3], nc[3], nd[3] = {0, 0, 0};
                cross3(qa, eab, m);                  /* = (a - o) x (b - o) */
                cross3(eab, eac, nc);
                if (ed[3] >= 0) cross3(eab, ead, nd);
                const double la = norm3(qa), leab = norm3(eab);
                /* FP32 error of (a - o) . (e1 x e2): the cross product of the
                 * edge vectors is off by at most 4 u |e1||e2| (inputs and
                 * roundings), a - o by u (|a - o| + |o|), the dot product by
                 * 3 u |a - o| |e1 x e2|: below (8 u |a - o| + u |o|) |e1||e2|;
                 * the band takes four times that */
                const double tc = (32.0 * u * la + 4.0 * u * olen) * leab * norm3(eac);
                const double td = (32.0 * u * la + 4.0 * u * olen) * leab * norm3(ead);
                const double eo = 32.0 * u * olen;   /* generous o error for the value bounds below */
                const double sc = dot3(qa, nc);
                const double sd = ed[3] >= 0 ? dot3(qa, nd) : 0.0;
                int flag = nov_near;
                if (fabs(sc) <= tc) flag = 1;
                if (ed[3] >= 0 && fabs(sd) <= td) flag = 1;
                if (sc == 0.0) continue;
                const int sil = ed[3] < 0 || !((sc > 0.0 && sd < 0.0) || (sc < 0.0 && sd > 0.0));
                if (!sil && !flag) continue;
                double w[3];
                for (int k = 0; k < 3; ++k) w[k] = qa[k] + t * eab[k];
                const double r2 = dot3(w, w), rr = sqrt(r2);
                for (int k = 0; k < 3; ++k) w[k] /= rr;
                const double NoL = dot3(S.n, w);
                /* bound on the FP32 error of the direction w (radians): a few
                 * roundings plus o's own rounding seen from distance r */
                const double wband = 16.0 * u + 4.0 * u * olen / rr;
                /* robustly below the horizon: no term, whatever else is undecided */
                const int nol_near = fabs(NoL) < wband;
                if (NoL <= 0.0 && !nol_near) continue;
                if (nol_near) flag = 1;
                const double ml = norm3(m);
                if (ml == 0.0) continue;
                double mh[3];
                for (int k = 0; k < 3; ++k) mh[k] = m[k] / ml;
                const double s = sc > 0.0 ? 1.0 : -1.0;
                double ex[3];
                cross3(eab, w, ex);
                const double J = norm3(ex) / r2;
                /* radiance at w */
                int ti, tj;
                double margin, x, y, Lv[3], dLv[3] = {0, 0, 0};
                texel_of_dir_xy(E->H, E->W, w, &ti, &tj, &margin, &x, &y);
                double Lb[3];
                if (P->flags & ORC_BILINEAR) {
                    orc_probe_bilinear(E->env, E->H, E->W, x, y, Lv);
                    /* coordinates from an FP32 direction: the arc error of w
                     * (16 u, doubled) through theta and phi, plus atan2 and scaling */
                    const double dw = 32.0 * u;
                    const double rho = sqrt(w[0] * w[0] + w[2] * w[2]);
                    double bdy = (dw + 8.0 * u * ORC_PI) * (double)E->H / ORC_PI + 4.0 * u * y;
                    double bdx = (rho > 0.0 ? dw / rho : (double)E->W) * (double)E->W / (2.0 * ORC_PI) +
                                 8.0 * u * (double)E->W + 4.0 * u * x;
                    bilinear_shift_bound(E->env, E->H, E->W, x, y, fmin(bdx, (double)E->W),
                                         fmin(bdy, (double)E->H), dLv);
                    for (int c = 0; c < 3; ++c) Lb[c] = fabs(Lv[c]) + dLv[c];
                } else {
                    const float* Lr = E->env + ((size_t)ti * E->W + tj) * 3;
                    for (int c = 0; c < 3; ++c) Lv[c] = (double)Lr[c];
                    if (margin < 2.0 * wband + 64.0 * u) {
                        flag = 1;
                        texel_max3(E->env, E->H, E->W, ti, tj, Lb);
                    } else {
                        for (int c = 0; c < 3; ++c) Lb[c] = fabs(Lv[c]);
                    }
                }
                /* integrand of c_d and c_s at w, unshadowed (unit density, one
                 * sample), contracted with the upstream gradients */
                double gsum = 0.0, gabs = 0.0, gcond = 0.0, gbound = 0.0;
                {
                    /* below or at the horizon and undecided: bound the terms
                     * by those of the highest direction the FP32 one can be
                     * (they vanish continuously at the horizon) */
                    double we[3];
                    const int above = NoL > 0.0;
                    for (int k = 0; k < 3; ++k) we[k] = above ? w[k] : w[k] + (wband - NoL) * S.n[k];
                    const double wel = norm3(we);
                    for (int k = 0; k < 3; ++k) we[k] /= wel;
                    if (above || flag) {
                        pix_out po;
                        env_contrib ec;
                        memset(&po, 0, sizeof(po));
                        eval_sample(&S, &S, 1.0f, we, 0.0, 0.0, Lv, dLv, 1, 1.0, 0, NULL, NULL, &po, &ec, 1.0, 0.0, 1);
                        for (int c = 0; c < 3; ++c) {
                            const double td = fabs(ud[c] * po.val[T_CD + c]) + fabs(us[c] * po.val[T_CS + c]);
                            const double sl = fabs(Lv[c]) > 0.0 ? Lb[c] / fabs(Lv[c]) : 0.0;
                            gbound += td * sl;
                            if (!above) continue;
                            gsum += ud[c] * po.val[T_CD + c] + us[c] * po.val[T_CS + c];
                            gabs += td;
                            gcond += fabs(ud[c]) * (po.cond[T_CD + c] + po.lerr[T_CD + c]) +
                                     fabs(us[c]) * (po.cond[T_CS + c] + po.lerr[T_CS + c]);
                        }
                        if (!above) gbound *= 2.0;
                    }
                }
                /* a pixel whose n.v sign is undecided may carry a specular
                 * term or not: twice the bound covers either */
                if (nov_near) gbound = 2.0 * gbound + gabs;
                /* FP32 relative error of the geometric factors: mh through |m|
                 * against |a - o||b - a|, J through |(b-a) x w| against |b-a|, the
                 * differences from the rounded o, and a few roundings */
                const double lex = norm3(ex);
                const double rel_geo = u * (16.0 + la * leab / ml + leab / fmax(lex, 1e-300)) +
                                       eo * (leab / ml + (4.0 + leab / fmax(lex, 1e-300)) / rr);
                /* undecided band of the out-side ray: o's FP32 rounding plus
                 * the direction's error (and the triangle test's rounding)
                 * times the distance along the ray */
                const double vis_abs = 8.0 * u * olen, vis_rel = 2.0 * wband + 32.0 * u;
                const double base = wcls * P->tau * J / (double)n_es;
                const double wt = s * base * gsum;
                const double wcond = base * (gcond + gabs * rel_geo);
                const double wflag = base * fmax(gbound, gabs) * (1.0 + rel_geo);
                int blocked = 1;
                if (sil && NoL > 0.0) {
                    c5[1]++;
                    if (wt != 0.0 && isfinite(wt)) {
                        double wo[3];
                        for (int k = 0; k < 3; ++k) wo[k] = w[k] - s * ORC_EDGE_DELTA * mh[k];
                        const double wl = norm3(wo);
                        for (int k = 0; k < 3; ++k) wo[k] /= wl;
                        const int h = orc_anyhit(scene, o, wo, vis_abs, vis_rel, P->brute);
                        c5[2]++;
                        if (h == TRI_NEAR) flag = 1;
                        blocked = h != TRI_MISS;
                        if (blocked) c5[3]++;
                    }
                }
                /* an undecided sample whose out-side rays (either side when
                 * the face's side itself is undecided) are robustly blocked
                 * adds nothing on either side of its undecided steps */
                if (flag) {
                    const int both = fabs(sc) <= tc;
                    int all_hit = 1;
                    for (int side = 0; side < (both ? 2 : 1) && all_hit; ++side) {
                        const double ss = side == 0 ? s : -s;
                        double wo[3];
                        for (int k = 0; k < 3; ++k) wo[k] = w[k] - ss * ORC_EDGE_DELTA * mh[k];
                        const double wl = norm3(wo);
                        for (int k = 0; k < 3; ++k) wo[k] /= wl;
                        all_hit = orc_anyhit(scene, o, wo, vis_abs, vis_rel, P->brute) == TRI_HIT;
                    }
                    if (all_hit) flag = 0;
                }
                if (flag) c5[4]++;
                const double fa = 1.0 - t, fb = t;
                for (int k = 0; k < 3; ++k) {
                    const size_t ia = 3 * (size_t)ed[0] + k, ib = 3 * (size_t)ed[1] + k;
                    if (!blocked) {
                        a_v[ia] += wt * fa * mh[k];
                        a_v[ib] += wt * fb * mh[k];
                        a_abs[ia] += fabs(wt * fa * mh[k]);
                        a_abs[ib] += fabs(wt * fb * mh[k]);
                        a_cond[ia] += wcond * fa * fabs(mh[k]);
                        a_cond[ib] += wcond * fb * fabs(mh[k]);
                    }
                    if (flag) {
                        a_flag[ia] += wflag * fa;
                        a_flag[ib] += wflag * fb;
                    }
                }
            }
        }
    }
    for (int tid = 0; tid < nt; ++tid) {
        const double* a = acc + (size_t)tid * 4 * nv3;
        for (size_t i = 0; i < nv3; ++i) {
            gv[i] += a[i];
            gv_abs[i] += a[nv3 + i];
            gv_cond[i] += a[2 * nv3 + i];
            gv_flag[i] += a[3 * nv3 + i];
        }
        for (int k = 0; k < 5; ++k) counts[k] += cnt[tid * 5 + k];
    }
    free(acc);
    free(cnt);
    free(cls);
    return 0;
}

/* class of each edge (1 = sharp), for the pin tests */
void orc_edge_sharp(const float* verts, const int32_t* edges, int64_t n_edges, int32_t* out)
{
    for (int64_t e = 0; e < n_edges; ++e) out[e] = edge_is_sharp(verts, edges + 4 * e);
}
