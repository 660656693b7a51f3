/* CPU oracle of the reconstruction step of the joint activity / scatter
 * estimation loop (TOF-OSEM with a Joseph projector), binary64.
 *
 * TEST INFRASTRUCTURE ONLY: nothing in the product path includes, links or
 * calls this file.  It shares no code with the HIP library.
 *
 * The paper estimates scatter iteratively: reconstruct the activity with the
 * current scatter estimate, simulate scatter from it, smooth, repeat (Methods,
 * "Unknown activity distribution, very limited simulation time"), with
 * TOF-OSEM (Hudson and Larkin 1994) in 1 iteration of 28 subsets per loop
 * iteration, and an attenuation sinogram from a forward projection of the
 * attenuation map (Methods, "Evaluation metrics").  The projector is not
 * specified; the readings here:
 *
 *  - Geometry.  Sinogram bins as the simulator bins coincidences: the LOR of
 *    (view, rad) joins the centres of the two crystals the simulator maps to
 *    that bin (azimuth 2 pi (c + 1/2) / n_crystals on the detection cylinder),
 *    and plane p lies at z = -L/2 + (p + 1) pitch / 2 (the mean of the two
 *    rings' centres: direct and oblique ring pairs are rebinned to the plane
 *    of their mean, as the simulator's plane = r1 + r2 does).  The image has
 *    n_plane slices, slice p at plane p's z, on the phantom's transaxial
 *    grid, so each plane's LORs see one slice (2D projection per plane).
 *  - Joseph's method (Joseph 1982): along the LOR's major axis, one sample per
 *    pixel column (row) at the column's centre, linear interpolation between
 *    the two pixels next to the crossing point along the minor axis (pixels
 *    outside the image count 0), weight = pixel size / |direction component
 *    on the major axis| (the path length per column).  The major axis is
 *    decided from the crystal indices, not from rounded direction components:
 *    the LOR of crystals a, b runs at angle pi q / (2 n) with q = (2 k + n)
 *    mod 2n, k = (a + b + 1) mod n, so x is the major axis when 2q <= n or
 *    2q >= 3n (x at exactly 45 degrees).
 *  - TOF.  The TOF coordinate of a point of the LOR is its signed distance s
 *    from the LOR's midpoint towards the crystal the simulator takes as the
 *    TOF-positive end, as the simulator's tau = (path_B - path_A) / 2 is for
 *    an annihilation there; bin j covers [(j - n_tof/2) w, (j + 1 - n_tof/2) w),
 *    and a sample at s adds to bin j with weight Phi((hi - s)/sigma) -
 *    Phi((lo - s)/sigma), the probability that s plus the Gaussian timing
 *    error falls in the bin, for bins within 5 sigma of s (0 beyond); with
 *    sigma = 0 the bin holding s gets 1.
 *  - OSEM: subsets of views, view v in subset v mod n_subsets, visited in
 *    order; per subset x_j <- x_j (P_s^T (m y / (m P_s x + a)))_j /
 *    (P_s^T m)_j, with m the multiplicative sinogram (attenuation, detector
 *    sensitivity) shared by all TOF bins, a the additive one (scatter);
 *    ratios with a non-positive denominator count 0, positive denominators
 *    below 1e-20 count as 1e-20 (so that counts in a bin the model holds
 *    empty cannot overflow binary32 arithmetic), and pixels the subset does
 *    not see (zero sensitivity) keep their value.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define PI_R 3.141592653589793

/* For each (view, rad) the crystal pair the simulator's sinogram mapping
 * sends there: a[v * n_rad + r] is the TOF-positive end, b the other; -1 if
 * no pair maps there.  Uses the simulator's own mapping (orc_lor). */
void orc_recon_lor_table(int32_t n_crystals, int32_t n_rad, int32_t* a, int32_t* b) {
  const int n_view = n_crystals / 2, half = (n_rad - 1) / 2;
  for (int i = 0; i < n_view * n_rad; ++i) a[i] = b[i] = -1;
  for (int c1 = 0; c1 < n_crystals; ++c1)
    for (int c2 = c1 + 1; c2 < n_crystals; ++c2) {
      int32_t view, rho, apos;
      orc_lor(n_crystals, c1, c2, &view, &rho, &apos);
      if (abs(rho) > half) continue;
      const int k = view * n_rad + rho + half;
      a[k] = apos ? c1 : c2;
      b[k] = apos ? c2 : c1;
    }
}

typedef struct {
  const orc_scanner* sc;
  const orc_sino* sn;
  const orc_phantom* pd;   /* transaxial grid: nx, ny, voxel_mm[0..1], lo_mm[0..1] */
  int32_t* a;
  int32_t* b;
  int mx;                  /* major axis of the LOR last taken by lor_of: 1 = x */
} geo_t;

static int geo_init(geo_t* g, const orc_scanner* sc, const orc_sino* sn, const orc_phantom* pd) {
  if (!sc || !sn || !pd || sc->n_crystals <= 0 || sc->n_crystals % 2 || sn->n_view != sc->n_crystals / 2 ||
      sn->n_plane != 2 * sc->n_rings - 1 || sn->n_rad % 2 == 0 || pd->nx <= 0 || pd->ny <= 0)
    return -1;
  g->sc = sc; g->sn = sn; g->pd = pd;
  g->a = (int32_t*)malloc(sizeof(int32_t) * (size_t)sn->n_view * (size_t)sn->n_rad);
  g->b = (int32_t*)malloc(sizeof(int32_t) * (size_t)sn->n_view * (size_t)sn->n_rad);
  if (!g->a || !g->b) { free(g->a); free(g->b); return -1; }
  orc_recon_lor_table(sc->n_crystals, sn->n_rad, g->a, g->b);
  return 0;
}

static void geo_free(geo_t* g) { free(g->a); free(g->b); }

/* LOR of bin (view, rad): midpoint m, unit direction u towards the
 * TOF-positive end; 0 if no crystal pair maps there. */
static int lor_of(geo_t* g, int view, int rad, double m[2], double u[2]) {
  const int k = view * g->sn->n_rad + rad;
  if (g->a[k] < 0) return 0;
  const double R = g->sc->radius_mm, n = g->sc->n_crystals;
  const double pa = 2.0 * PI_R * (g->a[k] + 0.5) / n, pb = 2.0 * PI_R * (g->b[k] + 0.5) / n;
  const double ax = R * cos(pa), ay = R * sin(pa), bx = R * cos(pb), by = R * sin(pb);
  m[0] = 0.5 * (ax + bx);
  m[1] = 0.5 * (ay + by);
  const double dx = ax - bx, dy = ay - by, len = sqrt(dx * dx + dy * dy);
  u[0] = dx / len;
  u[1] = dy / len;
  const int nc = g->sc->n_crystals, kk = (g->a[k] + g->b[k] + 1) % nc, q = (2 * kk + nc) % (2 * nc);
  g->mx = 2 * q <= nc || 2 * q >= 3 * nc;
  return 1;
}

/* Weight of TOF bin j for a point at TOF coordinate s (see the header). */
static double tof_weight(const orc_sino* sn, int j, double s) {
  const double w = sn->tof_bin_mm, lo = (j - 0.5 * sn->n_tof) * w, hi = lo + w;
  const double sg = sn->tof_sigma_mm;
  if (sg <= 0.0) return (s >= lo && s < hi) ? 1.0 : 0.0;
  if (hi < s - 5.0 * sg || lo > s + 5.0 * sg) return 0.0;
  return 0.5 * (erf((hi - s) / (sg * sqrt(2.0))) - erf((lo - s) / (sg * sqrt(2.0))));
}

/* One Joseph sample k of the LOR (m, u): the pixel pair and weights it reads
 * (p0 with w0, p1 with w1; an index of -1 reads 0), its TOF coordinate s and
 * path length dl.  Samples run over the columns (major axis x) or rows. */
typedef struct { int p0, p1; double w0, w1, s, dl; } sample_t;

static int n_samples(const geo_t* g) { return g->mx ? g->pd->nx : g->pd->ny; }

static void sample(const geo_t* g, const double m[2], const double u[2], int k, sample_t* o) {
  const orc_phantom* pd = g->pd;
  const int nx = pd->nx, ny = pd->ny;
  const double vx = pd->voxel_mm[0], vy = pd->voxel_mm[1], lox = pd->lo_mm[0], loy = pd->lo_mm[1];
  double f;
  int i0, n_minor;
  if (g->mx) {
    const double xc = lox + (k + 0.5) * vx;
    o->s = (xc - m[0]) / u[0];
    const double y = m[1] + o->s * u[1];
    f = (y - loy) / vy - 0.5;
    o->dl = vx / fabs(u[0]);
    n_minor = ny;
  } else {
    const double yc = loy + (k + 0.5) * vy;
    o->s = (yc - m[1]) / u[1];
    const double x = m[0] + o->s * u[0];
    f = (x - lox) / vx - 0.5;
    o->dl = vy / fabs(u[1]);
    n_minor = nx;
  }
  i0 = (int)floor(f);
  const double fr = f - i0;
  o->w0 = 1.0 - fr;
  o->w1 = fr;
  const int j0 = i0, j1 = i0 + 1;
  if (g->mx) {
    o->p0 = (j0 >= 0 && j0 < n_minor) ? j0 * nx + k : -1;
    o->p1 = (j1 >= 0 && j1 < n_minor) ? j1 * nx + k : -1;
  } else {
    o->p0 = (j0 >= 0 && j0 < n_minor) ? k * nx + j0 : -1;
    o->p1 = (j1 >= 0 && j1 < n_minor) ? k * nx + j1 : -1;
  }
}

static int in_subset(int view, int subset, int n_subsets) { return n_subsets <= 1 || view % n_subsets == subset; }

/* Forward projection of the subset's views: sino[(t * n_plane + p) * n_view
 * + v) * n_rad + r] for TOF (tof = 1), or without the TOF axis (tof = 0: the
 * plain line integral); bins of other views are left as they are. */
int orc_recon_project(const orc_scanner* sc, const orc_sino* sn, const orc_phantom* pd, const double* img,
                      double* sino, int tof, int subset, int n_subsets) {
  geo_t g;
  if (geo_init(&g, sc, sn, pd)) return -1;
  const int nv = sn->n_view, nr = sn->n_rad, np = sn->n_plane, nt = tof ? sn->n_tof : 1;
  const size_t npix = (size_t)pd->nx * (size_t)pd->ny, plane_bins = (size_t)nv * nr;
  for (int p = 0; p < np; ++p)
    for (int v = 0; v < nv; ++v) {
      if (!in_subset(v, subset, n_subsets)) continue;
      for (int r = 0; r < nr; ++r) {
        for (int t = 0; t < nt; ++t) sino[((size_t)t * np + p) * plane_bins + (size_t)v * nr + r] = 0.0;
        double m[2], u[2];
        if (!lor_of(&g, v, r, m, u)) continue;
        const double* im = img + (size_t)p * npix;
        const int ns = n_samples(&g);
        for (int k = 0; k < ns; ++k) {
          sample_t o;
          sample(&g, m, u, k, &o);
          const double val = (o.p0 >= 0 ? o.w0 * im[o.p0] : 0.0) + (o.p1 >= 0 ? o.w1 * im[o.p1] : 0.0);
          if (val == 0.0) continue;
          for (int t = 0; t < nt; ++t) {
            const double tw = tof ? tof_weight(sn, t, o.s) : 1.0;
            sino[((size_t)t * np + p) * plane_bins + (size_t)v * nr + r] += tw * o.dl * val;
          }
        }
      }
    }
  geo_free(&g);
  return 0;
}

/* Back projection (the transpose) of the subset's views into img
 * (overwritten). */
int orc_recon_backproject(const orc_scanner* sc, const orc_sino* sn, const orc_phantom* pd, const double* sino,
                          double* img, int tof, int subset, int n_subsets) {
  geo_t g;
  if (geo_init(&g, sc, sn, pd)) return -1;
  const int nv = sn->n_view, nr = sn->n_rad, np = sn->n_plane, nt = tof ? sn->n_tof : 1;
  const size_t npix = (size_t)pd->nx * (size_t)pd->ny, plane_bins = (size_t)nv * nr;
  memset(img, 0, sizeof(double) * npix * (size_t)np);
  for (int p = 0; p < np; ++p)
    for (int v = 0; v < nv; ++v) {
      if (!in_subset(v, subset, n_subsets)) continue;
      for (int r = 0; r < nr; ++r) {
        double m[2], u[2];
        if (!lor_of(&g, v, r, m, u)) continue;
        double* im = img + (size_t)p * npix;
        const int ns = n_samples(&g);
        for (int k = 0; k < ns; ++k) {
          sample_t o;
          sample(&g, m, u, k, &o);
          if (o.p0 < 0 && o.p1 < 0) continue;
          double acc = 0.0;
          for (int t = 0; t < nt; ++t) {
            const double tw = tof ? tof_weight(sn, t, o.s) : 1.0;
            acc += tw * sino[((size_t)t * np + p) * plane_bins + (size_t)v * nr + r];
          }
          acc *= o.dl;
          if (o.p0 >= 0) im[o.p0] += o.w0 * acc;
          if (o.p1 >= 0) im[o.p1] += o.w1 * acc;
        }
      }
    }
  geo_free(&g);
  return 0;
}

/* n_iter iterations of TOF-OSEM with n_subsets subsets, in place on img.
 * prompts and add: TOF sinograms; mult: without the TOF axis. */
int orc_recon_osem(const orc_scanner* sc, const orc_sino* sn, const orc_phantom* pd, const double* prompts,
                   const double* mult, const double* add, double* img, int n_iter, int n_subsets) {
  const size_t nb = (size_t)sn->n_tof * sn->n_plane * sn->n_view * sn->n_rad;
  const size_t inner = (size_t)sn->n_plane * sn->n_view * sn->n_rad;
  const size_t ni = (size_t)pd->nx * pd->ny * sn->n_plane;
  const int nr = sn->n_rad, nv = sn->n_view;
  double* fp = (double*)malloc(sizeof(double) * nb);
  double* back = (double*)malloc(sizeof(double) * ni);
  double* sens = (double*)malloc(sizeof(double) * ni);
  double* mt = (double*)malloc(sizeof(double) * nb);
  if (!fp || !back || !sens || !mt) { free(fp); free(back); free(sens); free(mt); return -1; }
  for (size_t i = 0; i < nb; ++i) mt[i] = mult[i % inner];
  int rc = 0;
  for (int it = 0; it < n_iter && !rc; ++it)
    for (int s = 0; s < n_subsets && !rc; ++s) {
      rc |= orc_recon_project(sc, sn, pd, img, fp, 1, s, n_subsets);
      for (size_t i = 0; i < nb; ++i) {
        const int v = (int)((i / nr) % nv);
        if (!in_subset(v, s, n_subsets)) { fp[i] = 0.0; continue; }
        const double den = mt[i] * fp[i] + add[i];
        fp[i] = den > 0.0 ? mt[i] * prompts[i] / (den > 1e-20 ? den : 1e-20) : 0.0;
      }
      rc |= orc_recon_backproject(sc, sn, pd, fp, back, 1, s, n_subsets);
      rc |= orc_recon_backproject(sc, sn, pd, mt, sens, 1, s, n_subsets);
      for (size_t j = 0; j < ni; ++j)
        if (sens[j] > 0.0) img[j] = img[j] * back[j] / sens[j];
    }
  free(fp); free(back); free(sens); free(mt);
  return rc;
}
