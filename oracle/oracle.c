/*
 * oracle.c -- slow, plain FP64 reference for the line-of-sight projector of
 * Barbey, Guennou & Auchere, "TomograPy" (Solar Physics), and for the small
 * 3-D convolution network used as a preconditioner.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may load this file's
 * library: only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header or constant with the HIP library.
 *
 * What it computes (Sec. "Single Spacecraft Static Tomography", Eq. lo):
 *   y_j = sum_i P_{j,i} e_i, where P_{j,i} is the length of line of sight j
 *   inside voxel i (the paper's indices are garbled; this is the reading in
 *   which j runs over detector pixels and i over voxels).
 * The lengths are found with Siddon's method (the paper's projector, Sec.
 * "Fast Parallelized Projector"): the parametric values at which the ray
 * crosses every x, y and z voxel plane inside the box are collected per axis,
 * merged into one increasing sequence (exactly equal values merged), and each
 * consecutive pair gives one segment whose voxel is the one holding the
 * segment's midpoint.  The transpose scatters the same lengths.
 *
 * A second, independent route (the per-voxel slab clip) computes the same
 * lengths directly from the plain definition, one voxel box at a time.
 *
 * Ray model (the paper gives only "WCS keywords define the observer and the
 * projector", Sec. "Instrument Independence"): a pinhole half-line from the
 * observer o with direction d = w + x u + y v, where (x, y) are gnomonic
 * tangent-plane coordinates of the pixel centre in radians,
 * x = (col - crpix0) cdelt0, y = (row - crpix1) cdelt1, pixel centres at
 * integer 0-based indices.  Points o + t d with t >= 0.  Lengths are in box
 * units.  Voxels are half-open [lo + k D, lo + (k+1) D).
 *
 * Optional obstacle (the opaque photosphere, Sec. "Solar Tomography"; the
 * projector's obstacle variant, Sec. "Fast Parallelized Projector"; line of
 * sight integration stops at the photosphere, Sec. "Performance"): a sphere
 * of centre c and radius R.  The line of sight is integrated over
 * 0 <= t < t_c only, t_c being where it enters the sphere's interior (t_c = 0
 * when the observer is on or inside the sphere; no limit when the line
 * never enters it, a tangent line included).
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC oracle.c -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ---------------------------------------------------------------- geometry */

typedef struct {
    int n[3];         /* voxels along x, y, z                         */
    double lo[3];     /* box lower corner                              */
    double hi[3];     /* box upper corner                              */
    double delta[3];  /* voxel side along each axis                    */
} ora_grid;

/* One view: 16 doubles per view in the flat table handed over by Python:
 * obs[3] w[3] u[3] v[3] cdelt[2] crpix[2]; and two ints ncol, nrow. */
typedef struct {
    double o[3], w[3], u[3], v[3], cdelt[2], crpix[2];
    int ncol, nrow;
} ora_view;

static ora_grid make_grid(const int *n, const double *lo, const double *hi)
{
    ora_grid g;
    for (int a = 0; a < 3; ++a) {
        g.n[a] = n[a];
        g.lo[a] = lo[a];
        g.hi[a] = hi[a];
        g.delta[a] = (hi[a] - lo[a]) / (double)n[a];
    }
    return g;
}

static ora_view make_view(const double *t16, const int *npix)
{
    ora_view v;
    for (int a = 0; a < 3; ++a) {
        v.o[a] = t16[a];
        v.w[a] = t16[3 + a];
        v.u[a] = t16[6 + a];
        v.v[a] = t16[9 + a];
    }
    v.cdelt[0] = t16[12];
    v.cdelt[1] = t16[13];
    v.crpix[0] = t16[14];
    v.crpix[1] = t16[15];
    v.ncol = npix[0];
    v.nrow = npix[1];
    return v;
}

/* Direction of the line of sight through pixel (col, row): gnomonic (TAN)
 * pinhole, d = w + x u + y v. */
static void ray_dir(const ora_view *v, int col, int row, double d[3])
{
    double x = ((double)col - v->crpix[0]) * v->cdelt[0];
    double y = ((double)row - v->crpix[1]) * v->cdelt[1];
    for (int a = 0; a < 3; ++a)
        d[a] = v->w[a] + x * v->u[a] + y * v->v[a];
}

static double norm3(const double d[3])
{
    return sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
}

/* Parametric interval [t_in, t_out] of the half-line inside the (half-open)
 * box.  Returns 0 if the ray misses. */
static int clip_box(const double o[3], const double d[3], const double lo[3],
                    const double hi[3], double *t_in, double *t_out)
{
    double tin = 0.0, tout = INFINITY;
    for (int a = 0; a < 3; ++a) {
        if (d[a] != 0.0) {
            double t1 = (lo[a] - o[a]) / d[a];
            double t2 = (hi[a] - o[a]) / d[a];
            double tl = t1 < t2 ? t1 : t2;
            double th = t1 < t2 ? t2 : t1;
            if (tl > tin) tin = tl;
            if (th < tout) tout = th;
        } else if (!(lo[a] <= o[a] && o[a] < hi[a])) {
            return 0;
        }
    }
    if (!(tout > tin)) return 0;
    *t_in = tin;
    *t_out = tout;
    return 1;
}

/* Where the half-line o + t d (t >= 0) enters the interior |p - c| < R of
 * the sphere sph = {cx, cy, cz, R}: 0 if o is inside or on the sphere,
 * INFINITY if the half-line never enters it.  Written from the closest approach
 * t* = -(o - c).d / d.d at distance h from the centre: the contact is
 * t* - sqrt((R^2 - h^2) / d.d), which needs no difference of two nearly
 * equal large numbers when the observer is far away. */
static double sphere_contact(const double o[3], const double d[3], const double *sph)
{
    double oc[3], dd = 0.0, od = 0.0, oo = 0.0;
    for (int a = 0; a < 3; ++a) {
        oc[a] = o[a] - sph[a];
        dd += d[a] * d[a];
        od += oc[a] * d[a];
        oo += oc[a] * oc[a];
    }
    const double r2 = sph[3] * sph[3];
    if (oo <= r2) return 0.0;
    if (od >= 0.0) return INFINITY; /* outside and moving away */
    double ts = -od / dd, h2 = 0.0;
    for (int a = 0; a < 3; ++a) {
        double p = oc[a] + ts * d[a];
        h2 += p * p;
    }
    if (h2 >= r2) return INFINITY; /* passes beside (or touches) the sphere */
    return ts - sqrt((r2 - h2) / dd);
}

/* ------------------------------------------------------------ Siddon walk */

/* Per-thread scratch for the crossing sets of one ray. */
typedef struct {
    double *set[3];
    double *merged;
    int cap[3];
    int mcap;
} ora_scratch;

static int scratch_init(ora_scratch *s, const ora_grid *g)
{
    int tot = 2;
    for (int a = 0; a < 3; ++a) {
        s->cap[a] = g->n[a] + 1;
        tot += s->cap[a];
        s->set[a] = (double *)malloc(sizeof(double) * (size_t)s->cap[a]);
        if (!s->set[a]) return -1;
    }
    s->mcap = tot;
    s->merged = (double *)malloc(sizeof(double) * (size_t)tot);
    return s->merged ? 0 : -1;
}

static void scratch_free(ora_scratch *s)
{
    for (int a = 0; a < 3; ++a) free(s->set[a]);
    free(s->merged);
}

/* Siddon's crossing set for one axis: parametric values of the planes
 * lo + k delta, k = 0..n, that fall strictly inside (t_in, t_out), listed in
 * increasing order. */
static int axis_crossings(const ora_grid *g, int a, double o, double d,
                          double t_in, double t_out, double *out)
{
    int cnt = 0;
    if (d == 0.0) return 0;
    int n = g->n[a];
    for (int j = 0; j <= n; ++j) {
        int k = d > 0.0 ? j : n - j; /* increasing t either way */
        double plane = g->lo[a] + (double)k * g->delta[a];
        double t = (plane - o) / d;
        if (t > t_in && t < t_out) out[cnt++] = t;
    }
    return cnt;
}

/* Merge of up to three increasing sequences plus the two end points, with
 * exactly equal values kept once.  Returns the merged length. */
static int merge_sets(double t_in, double t_out, double *const set[3],
                      const int cnt[3], double *out)
{
    int pos[3] = {0, 0, 0};
    int m = 0;
    out[m++] = t_in;
    for (;;) {
        int best = -1;
        double bv = INFINITY;
        for (int a = 0; a < 3; ++a)
            if (pos[a] < cnt[a] && set[a][pos[a]] < bv) {
                bv = set[a][pos[a]];
                best = a;
            }
        if (best < 0) break;
        for (int a = 0; a < 3; ++a) /* advance every set holding this value */
            if (pos[a] < cnt[a] && set[a][pos[a]] == bv) pos[a]++;
        if (bv != out[m - 1]) out[m++] = bv;
    }
    if (t_out != out[m - 1]) out[m++] = t_out;
    return m;
}

static int clampi(int v, int lo, int hi)
{
    return v < lo ? lo : (v > hi ? hi : v);
}

/* Segments of one ray: for each, the flat voxel index (x fastest) and the
 * length, up to the obstacle sph (or NULL).  Returns the number of segments
 * (0 if the ray misses); -1 if the output capacity is too small. */
static int trace(const ora_grid *g, const double o[3], const double d[3],
                 const double *sph, ora_scratch *s, int32_t *idx, double *len,
                 double *tlo, int cap)
{
    double t_in, t_out;
    if (!clip_box(o, d, g->lo, g->hi, &t_in, &t_out)) return 0;
    if (sph) { /* the line of sight ends at the obstacle */
        double tc = sphere_contact(o, d, sph);
        if (tc < t_out) t_out = tc;
        if (!(t_out > t_in)) return 0;
    }
    int cnt[3];
    for (int a = 0; a < 3; ++a)
        cnt[a] = axis_crossings(g, a, o[a], d[a], t_in, t_out, s->set[a]);
    int m = merge_sets(t_in, t_out, s->set, cnt, s->merged);
    double dn = norm3(d);
    int nseg = 0;
    for (int k = 0; k + 1 < m; ++k) {
        double ta = s->merged[k], tb = s->merged[k + 1];
        double tm = 0.5 * (ta + tb);
        int iv[3];
        for (int a = 0; a < 3; ++a) {
            double q = (o[a] + tm * d[a] - g->lo[a]) / g->delta[a];
            iv[a] = clampi((int)floor(q), 0, g->n[a] - 1);
        }
        if (nseg >= cap) return -1;
        idx[nseg] = (int32_t)(((int64_t)iv[2] * g->n[1] + iv[1]) * g->n[0] + iv[0]);
        len[nseg] = (tb - ta) * dn;
        if (tlo) tlo[nseg] = ta;
        ++nseg;
    }
    return nseg;
}

static int max_segments(const ora_grid *g)
{
    return g->n[0] + g->n[1] + g->n[2] + 3;
}

/* ------------------------------------------------------------ exported API */

/* Offsets of each view's first pixel in the concatenated image vector. */
static void view_offsets(int nviews, const int *npix, int64_t *off)
{
    int64_t acc = 0;
    for (int v = 0; v < nviews; ++v) {
        off[v] = acc;
        acc += (int64_t)npix[2 * v] * npix[2 * v + 1];
    }
    off[nviews] = acc;
}

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

int ora_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Projection P (and P M with a map mask M): images[ray] = sum of
 * length * cube[voxel] along the ray.  Masked pixels (data_mask == 0) are not
 * projected and give 0.  Views with view_frame[v] = f read frame f of a
 * cube holding nframes consecutive volumes (block-diagonal operator of the
 * smooth temporal model, Eq. srt_t).
 */
int ora_project(const int *n, const double *lo, const double *hi, int nviews,
                const double *views, const int *npix, const int *view_frame,
                const uint8_t *data_mask, const uint8_t *map_mask,
                const double *obstacle, const double *cube, double *images, int nthreads)
{
    ora_grid g = make_grid(n, lo, hi);
    int64_t nvox = (int64_t)n[0] * n[1] * n[2];
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nviews + 1));
    if (!off) return -1;
    view_offsets(nviews, npix, off);
    set_threads(nthreads);
    int err = 0;
    for (int v = 0; v < nviews; ++v) {
        ora_view vw = make_view(views + 16 * v, npix + 2 * v);
        const double *x = cube + (view_frame ? (int64_t)view_frame[v] * nvox : 0);
        const uint8_t *mm = map_mask;
        int64_t nray = (int64_t)vw.ncol * vw.nrow;
#pragma omp parallel
        {
            ora_scratch s;
            int cap = max_segments(&g);
            int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
            double *len = (double *)malloc(sizeof(double) * (size_t)cap);
            if (scratch_init(&s, &g) || !idx || !len) {
#pragma omp atomic write
                err = -1;
            } else {
#pragma omp for schedule(dynamic, 64)
                for (int64_t r = 0; r < nray; ++r) {
                    int col = (int)(r % vw.ncol), row = (int)(r / vw.ncol);
                    double acc = 0.0;
                    if (!data_mask || data_mask[off[v] + r]) {
                        double d[3];
                        ray_dir(&vw, col, row, d);
                        int ns = trace(&g, vw.o, d, obstacle, &s, idx, len, NULL, cap);
                        for (int k = 0; k < ns; ++k)
                            if (!mm || mm[idx[k]]) acc += len[k] * x[idx[k]];
                    }
                    images[off[v] + r] = acc;
                }
            }
            scratch_free(&s);
            free(idx);
            free(len);
        }
    }
    free(off);
    return err;
}

/*
 * Transpose P^T (M P^T with a map mask): cube[voxel] += length * images[ray]
 * for every segment of every unmasked ray.  The cube is zeroed first unless
 * accumulate != 0.  Concurrent updates of one voxel use an atomic add, as in
 * the paper's multithreaded back-projection (Sec. "Performance").
 */
int ora_backproject(const int *n, const double *lo, const double *hi,
                    int nviews, const double *views, const int *npix,
                    const int *view_frame, int nframes,
                    const uint8_t *data_mask, const uint8_t *map_mask,
                    const double *obstacle, const double *images, double *cube,
                    int accumulate, int nthreads)
{
    ora_grid g = make_grid(n, lo, hi);
    int64_t nvox = (int64_t)n[0] * n[1] * n[2];
    if (!accumulate) memset(cube, 0, sizeof(double) * (size_t)(nvox * (nframes > 0 ? nframes : 1)));
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nviews + 1));
    if (!off) return -1;
    view_offsets(nviews, npix, off);
    set_threads(nthreads);
    int err = 0;
    for (int v = 0; v < nviews; ++v) {
        ora_view vw = make_view(views + 16 * v, npix + 2 * v);
        double *x = cube + (view_frame ? (int64_t)view_frame[v] * nvox : 0);
        const uint8_t *mm = map_mask;
        int64_t nray = (int64_t)vw.ncol * vw.nrow;
#pragma omp parallel
        {
            ora_scratch s;
            int cap = max_segments(&g);
            int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
            double *len = (double *)malloc(sizeof(double) * (size_t)cap);
            if (scratch_init(&s, &g) || !idx || !len) {
#pragma omp atomic write
                err = -1;
            } else {
#pragma omp for schedule(dynamic, 64)
                for (int64_t r = 0; r < nray; ++r) {
                    if (data_mask && !data_mask[off[v] + r]) continue;
                    double yv = images[off[v] + r];
                    int col = (int)(r % vw.ncol), row = (int)(r / vw.ncol);
                    double d[3];
                    ray_dir(&vw, col, row, d);
                    int ns = trace(&g, vw.o, d, obstacle, &s, idx, len, NULL, cap);
                    for (int k = 0; k < ns; ++k) {
                        if (mm && !mm[idx[k]]) continue;
                        double add = len[k] * yv;
#pragma omp atomic update
                        x[idx[k]] += add;
                    }
                }
            }
            scratch_free(&s);
            free(idx);
            free(len);
        }
    }
    free(off);
    return err;
}

/* Number of positive-length ray/voxel segments over all unmasked rays (the
 * voxel-crossing count).  Map masks do not change it: a masked voxel is still
 * crossed, its value is just treated as zero. */
int64_t ora_count_crossings(const int *n, const double *lo, const double *hi,
                            int nviews, const double *views, const int *npix,
                            const uint8_t *data_mask, const double *obstacle, int nthreads)
{
    ora_grid g = make_grid(n, lo, hi);
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nviews + 1));
    if (!off) return -1;
    view_offsets(nviews, npix, off);
    set_threads(nthreads);
    int64_t total = 0;
    int err = 0;
    for (int v = 0; v < nviews; ++v) {
        ora_view vw = make_view(views + 16 * v, npix + 2 * v);
        int64_t nray = (int64_t)vw.ncol * vw.nrow;
#pragma omp parallel
        {
            ora_scratch s;
            int cap = max_segments(&g);
            int32_t *idx = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
            double *len = (double *)malloc(sizeof(double) * (size_t)cap);
            if (scratch_init(&s, &g) || !idx || !len) {
#pragma omp atomic write
                err = -1;
            } else {
#pragma omp for schedule(dynamic, 64) reduction(+ : total)
                for (int64_t r = 0; r < nray; ++r) {
                    if (data_mask && !data_mask[off[v] + r]) continue;
                    int col = (int)(r % vw.ncol), row = (int)(r / vw.ncol);
                    double d[3];
                    ray_dir(&vw, col, row, d);
                    int ns = trace(&g, vw.o, d, obstacle, &s, idx, len, NULL, cap);
                    for (int k = 0; k < ns; ++k) total += len[k] > 0.0;
                }
            }
            scratch_free(&s);
            free(idx);
            free(len);
        }
    }
    free(off);
    return err ? -1 : total;
}

/* Segment list of one line of sight, given its origin and direction
 * directly (so tests can place hand-made rays), up to the obstacle (or
 * NULL).  tlo receives each segment's entry parameter.  Returns the segment
 * count or -1 on overflow. */
int ora_trace_ray(const int *n, const double *lo, const double *hi,
                  const double *o, const double *d, const double *obstacle,
                  int32_t *idx, double *len, double *tlo, int cap)
{
    ora_grid g = make_grid(n, lo, hi);
    ora_scratch s;
    if (scratch_init(&s, &g)) return -1;
    int ns = trace(&g, o, d, obstacle, &s, idx, len, tlo, cap);
    scratch_free(&s);
    return ns;
}

/* Direction of the ray through pixel (col, row) of one view. */
void ora_pixel_direction(const double *view16, const int *npix, int col,
                         int row, double *d)
{
    ora_view vw = make_view(view16, npix);
    ray_dir(&vw, col, row, d);
}

/*
 * Brute-force twin of one ray's row of P, straight from the definition:
 * for every voxel, clip the half-line against that voxel's own box and take
 * the length inside, up to the obstacle's first contact (obstacle may be
 * NULL).  O(voxels) per ray, no merging; only for tiny cubes.  out has one
 * entry per voxel (x fastest).
 */
void ora_ray_row_bruteforce(const int *n, const double *lo, const double *hi,
                            const double *o, const double *d, const double *obstacle,
                            double *out)
{
    ora_grid g = make_grid(n, lo, hi);
    double dn = norm3(d);
    double tc = obstacle ? sphere_contact(o, d, obstacle) : INFINITY;
    for (int k = 0; k < g.n[2]; ++k)
        for (int j = 0; j < g.n[1]; ++j)
            for (int i = 0; i < g.n[0]; ++i) {
                int iv[3] = {i, j, k};
                double vlo[3], vhi[3];
                for (int a = 0; a < 3; ++a) {
                    vlo[a] = g.lo[a] + (double)iv[a] * g.delta[a];
                    vhi[a] = g.lo[a] + (double)(iv[a] + 1) * g.delta[a];
                }
                double tin, tout;
                double l = 0.0;
                if (clip_box(o, d, vlo, vhi, &tin, &tout)) {
                    if (tc < tout) tout = tc;
                    if (tout > tin) l = (tout - tin) * dn;
                }
                out[((int64_t)k * g.n[1] + j) * g.n[0] + i] = l;
            }
}

/* ------------------------------------------------- 3-D convolution network */

/*
 * 3x3x3 convolution, stride 1, zero padding 1, cross-correlation convention
 * (the one torch uses).  in: [cin][nz][ny][nx]; w: [cout][cin][3][3][3];
 * b: [cout] or NULL; out: [cout][nz][ny][nx].
 */
void ora_conv3d_forward(int cin, int cout, int nz, int ny, int nx,
                        const double *in, const double *w, const double *b,
                        double *out)
{
    int64_t plane = (int64_t)ny * nx, vol = plane * nz;
#pragma omp parallel for collapse(2) schedule(static)
    for (int co = 0; co < cout; ++co)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    double acc = b ? b[co] : 0.0;
                    for (int ci = 0; ci < cin; ++ci)
                        for (int kz = 0; kz < 3; ++kz)
                            for (int ky = 0; ky < 3; ++ky)
                                for (int kx = 0; kx < 3; ++kx) {
                                    int zz = z + kz - 1, yy = y + ky - 1, xx = x + kx - 1;
                                    if (zz < 0 || zz >= nz || yy < 0 || yy >= ny || xx < 0 || xx >= nx)
                                        continue;
                                    acc += w[(((int64_t)co * cin + ci) * 3 + kz) * 9 + ky * 3 + kx] *
                                           in[ci * vol + zz * plane + (int64_t)yy * nx + xx];
                                }
                    out[co * vol + z * plane + (int64_t)y * nx + x] = acc;
                }
}

/* Gradient of the loss with respect to the convolution's input, given the
 * gradient with respect to its output. */
void ora_conv3d_backward_data(int cin, int cout, int nz, int ny, int nx,
                              const double *gout, const double *w, double *gin)
{
    int64_t plane = (int64_t)ny * nx, vol = plane * nz;
#pragma omp parallel for collapse(2) schedule(static)
    for (int ci = 0; ci < cin; ++ci)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    double acc = 0.0;
                    /* out[co][z'] uses in[ci][z' + k - 1]; here z = z' + k - 1 */
                    for (int co = 0; co < cout; ++co)
                        for (int kz = 0; kz < 3; ++kz)
                            for (int ky = 0; ky < 3; ++ky)
                                for (int kx = 0; kx < 3; ++kx) {
                                    int zo = z - kz + 1, yo = y - ky + 1, xo = x - kx + 1;
                                    if (zo < 0 || zo >= nz || yo < 0 || yo >= ny || xo < 0 || xo >= nx)
                                        continue;
                                    acc += w[(((int64_t)co * cin + ci) * 3 + kz) * 9 + ky * 3 + kx] *
                                           gout[co * vol + zo * plane + (int64_t)yo * nx + xo];
                                }
                    gin[ci * vol + z * plane + (int64_t)y * nx + x] = acc;
                }
}

/* Gradients with respect to the weights and the bias. */
void ora_conv3d_backward_weight(int cin, int cout, int nz, int ny, int nx,
                                const double *in, const double *gout,
                                double *gw, double *gb)
{
    int64_t plane = (int64_t)ny * nx, vol = plane * nz;
#pragma omp parallel for collapse(2) schedule(static)
    for (int co = 0; co < cout; ++co)
        for (int ci = 0; ci < cin; ++ci)
            for (int kz = 0; kz < 3; ++kz)
                for (int ky = 0; ky < 3; ++ky)
                    for (int kx = 0; kx < 3; ++kx) {
                        double acc = 0.0;
                        for (int z = 0; z < nz; ++z)
                            for (int y = 0; y < ny; ++y)
                                for (int x = 0; x < nx; ++x) {
                                    int zz = z + kz - 1, yy = y + ky - 1, xx = x + kx - 1;
                                    if (zz < 0 || zz >= nz || yy < 0 || yy >= ny || xx < 0 || xx >= nx)
                                        continue;
                                    acc += gout[co * vol + z * plane + (int64_t)y * nx + x] *
                                           in[ci * vol + zz * plane + (int64_t)yy * nx + xx];
                                }
                        gw[(((int64_t)co * cin + ci) * 3 + kz) * 9 + ky * 3 + kx] = acc;
                    }
    if (gb)
        for (int co = 0; co < cout; ++co) {
            double acc = 0.0;
            for (int64_t i = 0; i < vol; ++i) acc += gout[co * vol + i];
            gb[co] = acc;
        }
}
