/*
 * fov_oracle.c -- FP64 CPU oracle for block-wise foveation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library calls, links or
 * includes this file; only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header, table or
 * constant with the HIP path.
 *
 * What it computes (Malkin, Deza, Poggio, "CUDA-Optimized real-time rendering
 * of a Foveated Visual System", arXiv 2012.08655):
 *
 *   - The frame is cut into square fragments of side B; every fragment is
 *     blurred with one Gaussian whose strength follows the distance from the
 *     fragment midpoint to the fixation point (Sec. 2 "Block-wise Foveation",
 *     Fig. 1; Appendix "Workload of the Block").
 *   - The Gaussian is Eq. (1), sampled at integer offsets around the centre
 *     tap, cut off beyond 3 sigma and normalised to sum 1 (Appendix
 *     "Methods", text after Eq. 1).  Radius r = ceil(3 sigma), N = 2r+1 taps.
 *   - A foveal fragment (sigma = 0) is copied unchanged (Appendix "Workload
 *     of the Block").
 *
 * The oracle evaluates the plain, NON-separable 2-D definition
 *     out(y,x) = sum_{i,j=-r..r} G(i,j) / S * in(clamp(y+i), clamp(x+j)),
 *     S = sum_{i,j} G(i,j),   G from Eq. (1)
 * directly, in double precision, with clamp-to-edge indexing.  The paper's
 * separable H-then-V pass (Appendix "Methods", Fig. 9) is a faster way to
 * reach the same linear map; it is NOT used here.
 *
 * Readings of points the paper leaves open (listed with the same numbers in
 * the design notes):
 *   c1  window: r = ceil(3 sigma), N = 2r+1 taps centred on the pixel.
 *   c2  fragment midpoint in pixel-centre coordinates:
 *       c = origin + b*B + (B-1)/2, (0,0) is the centre of the top-left pixel.
 *   c3  partial edge fragments use their nominal (unclipped) midpoint.
 *   c4  outside the frame: clamp-to-edge, per axis.
 *   c5  sigma(e) = 0 for e < e0, else min(slope*(e-e0), cap); any fragment
 *       with sigma = 0 is copied.
 *   c6  sigma and r in IEEE double, no contraction, in the order written.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (see oracle.py).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double fix_x, fix_y; /* fixation, pixel-centre coordinates */
    double e0;           /* eccentricity (px) below which a fragment is foveal */
    double slope;        /* sigma growth per px of eccentricity beyond e0 */
    double cap;          /* largest sigma */
    int32_t block;       /* fragment side B */
    int32_t origin_x;    /* x of the left edge of fragment column 0, in (-B, 0] */
    int32_t origin_y;    /* y of the top edge of fragment row 0, in (-B, 0] */
} orc_frame;

static int floordiv(int a, int b) { /* b > 0 */
    int q = a / b;
    if ((a % b) != 0 && ((a < 0) != (b < 0))) q -= 1;
    return q;
}

static int clampi(int v, int lo, int hi) { return v < lo ? lo : (v > hi ? hi : v); }

/* Number of fragment columns / rows that cover a w x h frame. */
void orc_grid(int h, int w, const orc_frame* f, int32_t* nbx, int32_t* nby)
{
    int B = f->block;
    *nbx = floordiv(w - 1 - f->origin_x, B) + 1;
    *nby = floordiv(h - 1 - f->origin_y, B) + 1;
}

/*
 * Blur strength of fragment (bx, by): distance from the fragment midpoint to
 * the fixation (Sec. 2, Fig. 1), mapped through the eccentricity ramp (c5).
 * With a sigma map (Sec. 4 "Discussion": any image may give the blurring
 * strength), the map value replaces the ramp and is clipped to [0, cap].
 */
static double orc_sigma(const orc_frame* f, int bx, int by, int nbx, const double* sigma_map)
{
    double sigma;
    if (sigma_map) {
        double m = sigma_map[(size_t)by * nbx + bx];
        if (!(m > 0.0)) return 0.0;
        sigma = m < f->cap ? m : f->cap;
        return sigma > 0.0 ? sigma : 0.0;
    }
    double half = (double)(f->block - 1) / 2.0;
    double cx = (double)f->origin_x + (double)bx * (double)f->block + half;
    double cy = (double)f->origin_y + (double)by * (double)f->block + half;
    double dx = cx - f->fix_x;
    double dy = cy - f->fix_y;
    double e = sqrt(dx * dx + dy * dy);
    if (e < f->e0) return 0.0;
    sigma = f->slope * (e - f->e0);
    if (sigma > f->cap) sigma = f->cap;
    return sigma > 0.0 ? sigma : 0.0;
}

/* Truncation radius: values beyond 3 sigma are dropped (Appendix "Methods"). */
static int orc_radius(double sigma)
{
    if (!(sigma > 0.0)) return 0;
    return (int)ceil(3.0 * sigma);
}

/* Per-fragment plan: sigma and radius for every fragment, row-major. */
void orc_plan(int h, int w, const orc_frame* f, const double* sigma_map,
              double* sigma_out, int32_t* r_out)
{
    int32_t nbx, nby;
    orc_grid(h, w, f, &nbx, &nby);
    for (int by = 0; by < nby; ++by)
        for (int bx = 0; bx < nbx; ++bx) {
            double s = orc_sigma(f, bx, by, nbx, sigma_map);
            sigma_out[(size_t)by * nbx + bx] = s;
            r_out[(size_t)by * nbx + bx] = orc_radius(s);
        }
}

/*
 * Normalised 2-D Gaussian window of Eq. (1) on the (2r+1)^2 integer grid:
 * G(i,j) = exp(-(i^2+j^2) / (2 sigma^2)) / (2 pi sigma^2), divided by the sum
 * of all its taps.  (The 1/(2 pi sigma^2) factor cancels in the
 * normalisation and is kept only so the code reads as the equation.)
 * Returns a malloc'd (2r+1)^2 array, row index i, column index j.
 */
static double* orc_window2d(double sigma, int r)
{
    int n = 2 * r + 1;
    double* g = (double*)malloc(sizeof(double) * (size_t)n * n);
    if (r == 0) { g[0] = 1.0; return g; }
    double norm = 1.0 / (2.0 * M_PI * sigma * sigma);
    double s = 0.0;
    for (int i = -r; i <= r; ++i)
        for (int j = -r; j <= r; ++j) {
            double v = norm * exp(-((double)(i * i + j * j)) / (2.0 * sigma * sigma));
            g[(size_t)(i + r) * n + (j + r)] = v;
            s += v;
        }
    for (int k = 0; k < n * n; ++k) g[k] /= s;
    return g;
}

/* Output pixel (y, x) of one channel plane: the direct 2-D sum with clamp. */
static double orc_pixel(const double* plane, int h, int w, int y, int x,
                        const double* g, int r)
{
    if (r == 0) return plane[(size_t)y * w + x];
    int n = 2 * r + 1;
    double acc = 0.0;
    for (int i = -r; i <= r; ++i) {
        const double* row = plane + (size_t)clampi(y + i, 0, h - 1) * w;
        const double* gr = g + (size_t)(i + r) * n + r;
        for (int j = -r; j <= r; ++j) acc += gr[j] * row[clampi(x + j, 0, w - 1)];
    }
    return acc;
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
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

/*
 * Forward map of one frame: in/out are contiguous [c][h][w] double planes.
 * Parallel over fragments; each output is computed independently.
 */
void orc_forward(const double* in, double* out, int c, int h, int w,
                 const orc_frame* f, const double* sigma_map, int nthreads)
{
    int32_t nbx, nby;
    orc_grid(h, w, f, &nbx, &nby);
    set_threads(nthreads);
    int nblk = nbx * nby;
#pragma omp parallel for schedule(dynamic, 1)
    for (int b = 0; b < nblk; ++b) {
        int bx = b % nbx, by = b / nbx;
        double sigma = orc_sigma(f, bx, by, nbx, sigma_map);
        int r = orc_radius(sigma);
        double* g = orc_window2d(sigma, r);
        int x0 = f->origin_x + bx * f->block, y0 = f->origin_y + by * f->block;
        int xa = x0 < 0 ? 0 : x0, ya = y0 < 0 ? 0 : y0;
        int xb = x0 + f->block > w ? w : x0 + f->block;
        int yb = y0 + f->block > h ? h : y0 + f->block;
        for (int ch = 0; ch < c; ++ch) {
            const double* plane = in + (size_t)ch * h * w;
            double* oplane = out + (size_t)ch * h * w;
            for (int y = ya; y < yb; ++y)
                for (int x = xa; x < xb; ++x)
                    oplane[(size_t)y * w + x] = orc_pixel(plane, h, w, y, x, g, r);
        }
        free(g);
    }
}

/*
 * Forward map evaluated only at the listed pixels (for sampled checks of
 * large frames).  out is [npts][c].
 */
void orc_forward_points(const double* in, int c, int h, int w, const orc_frame* f,
                        const double* sigma_map, const int32_t* ys, const int32_t* xs,
                        int npts, double* out, int nthreads)
{
    int32_t nbx, nby;
    orc_grid(h, w, f, &nbx, &nby);
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 4)
    for (int k = 0; k < npts; ++k) {
        int y = ys[k], x = xs[k];
        int bx = floordiv(x - f->origin_x, f->block);
        int by = floordiv(y - f->origin_y, f->block);
        double sigma = orc_sigma(f, bx, by, nbx, sigma_map);
        int r = orc_radius(sigma);
        double* g = orc_window2d(sigma, r);
        for (int ch = 0; ch < c; ++ch)
            out[(size_t)k * c + ch] = orc_pixel(in + (size_t)ch * h * w, h, w, y, x, g, r);
        free(g);
    }
}

/*
 * "Perfect" foveation, the reference of the paper's quality comparison (Sec. 3,
 * Fig. 3): every pixel is blurred with its own sigma, from its own distance to
 * the fixation (pixel-centre coordinates) through the same ramp, instead of
 * its fragment midpoint's.  The window is Eq. (1) normalised over the square
 * (2r+1)^2 grid, i.e. the outer product of the normalised 1-D taps g, and the
 * sum is taken row by row: out = sum_i g(i) sum_j g(j) in(clamp(y+i), clamp(x+j)).
 * The tiling fields of f (block, origin) and the sigma map do not apply.
 */
void orc_forward_per_pixel(const double* in, double* out, int c, int h, int w, const orc_frame* f, int nthreads)
{
    set_threads(nthreads);
#pragma omp parallel for schedule(dynamic, 1)
    for (int y = 0; y < h; ++y) {
        double* g = NULL;
        int gcap = 0;
        for (int x = 0; x < w; ++x) {
            double dx = (double)x - f->fix_x, dy = (double)y - f->fix_y;
            double e = sqrt(dx * dx + dy * dy);
            double sigma = 0.0;
            if (!(e < f->e0)) {
                sigma = f->slope * (e - f->e0);
                if (sigma > f->cap) sigma = f->cap;
                if (!(sigma > 0.0)) sigma = 0.0;
            }
            int r = orc_radius(sigma);
            if (r == 0) {
                for (int ch = 0; ch < c; ++ch)
                    out[((size_t)ch * h + y) * w + x] = in[((size_t)ch * h + y) * w + x];
                continue;
            }
            int n = 2 * r + 1;
            if (n > gcap) {
                free(g);
                g = (double*)malloc(sizeof(double) * (size_t)n);
                gcap = n;
            }
            double s = 0.0;
            for (int i = -r; i <= r; ++i) {
                g[i + r] = exp(-((double)(i * i)) / (2.0 * sigma * sigma));
                s += g[i + r];
            }
            for (int i = 0; i < n; ++i) g[i] /= s;
            for (int ch = 0; ch < c; ++ch) {
                const double* plane = in + (size_t)ch * h * w;
                double acc = 0.0;
                for (int i = -r; i <= r; ++i) {
                    const double* row = plane + (size_t)clampi(y + i, 0, h - 1) * w;
                    double racc = 0.0;
                    for (int j = -r; j <= r; ++j) racc += g[j + r] * row[clampi(x + j, 0, w - 1)];
                    acc += g[i + r] * racc;
                }
                out[((size_t)ch * h + y) * w + x] = acc;
            }
        }
        free(g);
    }
}

/*
 * Adjoint (transpose) of the forward map, by its definition
 *     (A^T g)(q) = sum_p A(p, q) g(p):
 * every output pixel p scatters g(p) * W(i,j) onto the clamped input pixel it
 * read.  Serial per channel plane so the scatter has no races.
 */
void orc_adjoint(const double* g, double* gin, int c, int h, int w,
                 const orc_frame* f, const double* sigma_map, int nthreads)
{
    int32_t nbx, nby;
    orc_grid(h, w, f, &nbx, &nby);
    set_threads(nthreads);
    memset(gin, 0, sizeof(double) * (size_t)c * h * w);
#pragma omp parallel for schedule(static, 1)
    for (int ch = 0; ch < c; ++ch) {
        const double* gp = g + (size_t)ch * h * w;
        double* op = gin + (size_t)ch * h * w;
        for (int by = 0; by < nby; ++by)
            for (int bx = 0; bx < nbx; ++bx) {
                double sigma = orc_sigma(f, bx, by, nbx, sigma_map);
                int r = orc_radius(sigma);
                double* win = orc_window2d(sigma, r);
                int n = 2 * r + 1;
                int x0 = f->origin_x + bx * f->block, y0 = f->origin_y + by * f->block;
                int xa = x0 < 0 ? 0 : x0, ya = y0 < 0 ? 0 : y0;
                int xb = x0 + f->block > w ? w : x0 + f->block;
                int yb = y0 + f->block > h ? h : y0 + f->block;
                for (int y = ya; y < yb; ++y)
                    for (int x = xa; x < xb; ++x) {
                        double gv = gp[(size_t)y * w + x];
                        for (int i = -r; i <= r; ++i) {
                            double* orow = op + (size_t)clampi(y + i, 0, h - 1) * w;
                            for (int j = -r; j <= r; ++j)
                                orow[clampi(x + j, 0, w - 1)] += win[(size_t)(i + r) * n + (j + r)] * gv;
                        }
                    }
                free(win);
            }
    }
}

/*
 * Eq. (7): bytes of on-chip shared memory one fragment needs -- a u8 tile of
 * tileW x tileH (fragment plus padding) and an f32 intermediate of
 * fragmentW x tileH.  With tile = fragment + N - 1 (padding of r on each side).
 */
long orc_eq7_shared_bytes(int frag, int n_taps)
{
    long tile = (long)frag + n_taps - 1;
    return tile * tile + 4L * frag * tile;
}
