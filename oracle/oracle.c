/*
 * oracle.c -- plain, slow FP64 CPU reference of the PIV hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Tests, the smoke check and the benchmark's
 * CPU-baseline leg call it; the product library neither links nor calls it,
 * and it shares no code, header or constant table with the GPU path.
 *
 * Every function below follows the method's steps literally, one window
 * (or node, or vector) at a time, with no sharing of partial sums between
 * windows and no fusion.  OpenMP only splits the outer loop over
 * independent windows/nodes; it does not change any arithmetic.
 *
 * Conventions (the paper gives no grid; these are this implementation's):
 *  - pixel (row i, col j) has its centre at x = j, y = i; intensity outside
 *    the image is 0;
 *  - the vector grid has nx = W/step, ny = H/step nodes; node (a, b) sits at
 *    (b*step + (step-1)/2, a*step + (step-1)/2) and its win x win window
 *    starts at b*step - (win-step)/2 (and likewise in y);
 *  - fields are [2][ny][nx] (u plane, then v plane), displacement from A to B.
 *
 * Paper references are to "RapidPIV: Full Flow-Field kHz PIV for Real-Time
 * Display and Control" (Bollt, Foxman, Gharib).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* per-vector flag bits (the values of the public flag enum, restated) */
enum { OF_FLAT = 1, OF_BORDER = 2, OF_NOCURV = 4, OF_OUTLIER = 8, OF_REPLACED = 16,
       OF_UNRESOLVED = 32 };

static int32_t ipx(const int32_t* I, int W, int H, int y, int x) {
  if (x < 0 || y < 0 || x >= W || y >= H) return 0;
  return I[(size_t)y * W + x];
}

static double dpx(const double* I, int W, int H, int y, int x) {
  if (x < 0 || y < 0 || x >= W || y >= H) return 0.0;
  return I[(size_t)y * W + x];
}

/* ------------------------------------------------------------------------
 * Predictor (replaces the optical-flow engine of Sec. 2, "RapidPIV": the
 * first, coarse estimate of the displacement field that the correlation
 * stage then corrects).  Coarse-to-fine integer block matching.
 * ---------------------------------------------------------------------- */

/* One pyramid level: out(y,x) = floor((I(2y,2x)+I(2y,2x+1)+I(2y+1,2x)+I(2y+1,2x+1)+2)/4),
 * with zero outside the input.  out is ceil(H/2) x ceil(W/2). */
void o_pyr_down(const int32_t* in, int W, int H, int32_t* out) {
  int W2 = (W + 1) / 2, H2 = (H + 1) / 2;
  for (int y = 0; y < H2; ++y)
    for (int x = 0; x < W2; ++x) {
      int32_t s = ipx(in, W, H, 2 * y, 2 * x) + ipx(in, W, H, 2 * y, 2 * x + 1) +
                  ipx(in, W, H, 2 * y + 1, 2 * x) + ipx(in, W, H, 2 * y + 1, 2 * x + 1);
      out[(size_t)y * W2 + x] = (s + 2) / 4; /* s >= 0: integer division is floor */
    }
}

/* Is (s1,l1,dy1,dx1) lexicographically smaller than (s2,l2,dy2,dx2)? */
static int key_less(int64_t s1, int l1, int dy1, int dx1, int64_t s2, int l2, int dy2, int dx2) {
  if (s1 != s2) return s1 < s2;
  if (l1 != l2) return l1 < l2;
  if (dy1 != dy2) return dy1 < dy2;
  return dx1 < dx2;
}

/* Integer SAD block search on one level.  For node (a,b) the block is
 * block x block pixels starting at (a*step + (step-block)/2, b*step + (step-block)/2);
 * SAD(d) = sum |A(q) - B(q+d)| over the block for d in cand + [-R,R]^2; the
 * chosen d minimises (SAD, |dx|+|dy|, dy, dx) lexicographically.
 * cand is [2][ny][nx] (NULL = zero); d is [2][ny][nx]. */
void o_sad_level(const int32_t* A, const int32_t* B, int W, int H, int nx, int ny, int step,
                 int block, int R, const int32_t* cand, int32_t* d) {
  int off = (step - block) / 2;
#pragma omp parallel for schedule(dynamic)
  for (int a = 0; a < ny; ++a)
    for (int b = 0; b < nx; ++b) {
      int oy = a * step + off, ox = b * step + off;
      int cx = cand ? cand[(size_t)a * nx + b] : 0;
      int cy = cand ? cand[(size_t)nx * ny + (size_t)a * nx + b] : 0;
      int64_t bs = -1;
      int bl = 0, bdy = 0, bdx = 0;
      for (int dy = cy - R; dy <= cy + R; ++dy)
        for (int dx = cx - R; dx <= cx + R; ++dx) {
          int64_t s = 0;
          for (int i = 0; i < block; ++i)
            for (int j = 0; j < block; ++j)
              s += llabs((long long)ipx(A, W, H, oy + i, ox + j) -
                         (long long)ipx(B, W, H, oy + i + dy, ox + j + dx));
          int l = abs(dx) + abs(dy);
          if (bs < 0 || key_less(s, l, dy, dx, bs, bl, bdy, bdx)) {
            bs = s; bl = l; bdy = dy; bdx = dx;
          }
        }
      d[(size_t)a * nx + b] = bdx;
      d[(size_t)nx * ny + (size_t)a * nx + b] = bdy;
    }
}

static int cmp_i32(const void* p, const void* q) {
  int32_t a = *(const int32_t*)p, b = *(const int32_t*)q;
  return (a > b) - (a < b);
}

/* 3x3 component-wise median over the in-bounds neighbourhood (centre
 * included); for an even count the lower of the two middle values. */
void o_median3_int(const int32_t* d, int nx, int ny, int32_t* out) {
  for (int c = 0; c < 2; ++c)
    for (int a = 0; a < ny; ++a)
      for (int b = 0; b < nx; ++b) {
        int32_t v[9];
        int k = 0;
        for (int i = a - 1; i <= a + 1; ++i)
          for (int j = b - 1; j <= b + 1; ++j)
            if (i >= 0 && j >= 0 && i < ny && j < nx)
              v[k++] = d[(size_t)c * nx * ny + (size_t)i * nx + j];
        qsort(v, k, sizeof(int32_t), cmp_i32);
        out[(size_t)c * nx * ny + (size_t)a * nx + b] = v[(k - 1) / 2];
      }
}

/* The whole predictor: pyramids, coarsest search with radius Rc around 0,
 * then per finer level a search with radius Rf around twice the parent
 * node's result, a 3x3 median after every level when `median` is set.
 * Level grids: nx_0 = W/step, nx_l = ceil(nx_{l-1}/2); level-l node (a,b)
 * has parent (a/2, b/2).  pred is [2][ny][nx] integers in level-0 pixels. */
void o_sgm_level(const int32_t* A, const int32_t* B, int W, int H, int nx, int ny, int step, int block, int R,
                 int p1, int p2, int32_t* d);

/* The predictor with the coarsest level searched by semi-global matching
 * (sgm != 0, penalties p1, p2 per block pixel) instead of block matching. */
void o_predict_sgm(const int32_t* A, const int32_t* B, int W, int H, int step, int block, int levels,
                   int Rc, int Rf, int median, int sgm, int p1, int p2, int32_t* pred);

void o_predict(const int32_t* A, const int32_t* B, int W, int H, int step, int block, int levels,
               int Rc, int Rf, int median, int32_t* pred) {
  o_predict_sgm(A, B, W, H, step, block, levels, Rc, Rf, median, 0, 0, 0, pred);
}

void o_predict_sgm(const int32_t* A, const int32_t* B, int W, int H, int step, int block, int levels,
                   int Rc, int Rf, int median, int sgm, int p1, int p2, int32_t* pred) {
  int Wl[16], Hl[16], nxl[16], nyl[16];
  const int32_t* PA[16];
  const int32_t* PB[16];
  int32_t* own[32];
  int nown = 0;
  Wl[0] = W; Hl[0] = H; nxl[0] = W / step; nyl[0] = H / step;
  PA[0] = A; PB[0] = B;
  for (int l = 1; l < levels; ++l) {
    Wl[l] = (Wl[l - 1] + 1) / 2; Hl[l] = (Hl[l - 1] + 1) / 2;
    nxl[l] = (nxl[l - 1] + 1) / 2; nyl[l] = (nyl[l - 1] + 1) / 2;
    int32_t* a = (int32_t*)malloc(sizeof(int32_t) * (size_t)Wl[l] * Hl[l]);
    int32_t* b = (int32_t*)malloc(sizeof(int32_t) * (size_t)Wl[l] * Hl[l]);
    o_pyr_down(PA[l - 1], Wl[l - 1], Hl[l - 1], a);
    o_pyr_down(PB[l - 1], Wl[l - 1], Hl[l - 1], b);
    PA[l] = a; PB[l] = b; own[nown++] = a; own[nown++] = b;
  }
  int32_t* prev = NULL;
  for (int l = levels - 1; l >= 0; --l) {
    int nx = nxl[l], ny = nyl[l];
    size_t np = (size_t)nx * ny;
    int32_t* cand = NULL;
    if (prev) {
      int pnx = nxl[l + 1], pny = nyl[l + 1];
      cand = (int32_t*)malloc(sizeof(int32_t) * 2 * np);
      for (int a = 0; a < ny; ++a)
        for (int b = 0; b < nx; ++b) {
          int pa = a / 2 < pny ? a / 2 : pny - 1, pb = b / 2 < pnx ? b / 2 : pnx - 1;
          for (int c = 0; c < 2; ++c)
            cand[c * np + (size_t)a * nx + b] = 2 * prev[(size_t)c * pnx * pny + (size_t)pa * pnx + pb];
        }
    }
    int32_t* d = (int32_t*)malloc(sizeof(int32_t) * 2 * np);
    if (sgm && l == levels - 1)
      o_sgm_level(PA[l], PB[l], Wl[l], Hl[l], nx, ny, step, block, Rc, p1, p2, d);
    else
      o_sad_level(PA[l], PB[l], Wl[l], Hl[l], nx, ny, step, block, l == levels - 1 ? Rc : Rf, cand, d);
    if (median) {
      int32_t* m = (int32_t*)malloc(sizeof(int32_t) * 2 * np);
      o_median3_int(d, nx, ny, m);
      free(d);
      d = m;
    }
    free(cand);
    free(prev);
    prev = d;
  }
  memcpy(pred, prev, sizeof(int32_t) * 2 * (size_t)nxl[0] * nyl[0]);
  free(prev);
  for (int i = 0; i < nown; ++i) free(own[i]);
}

/* ------------------------------------------------------------------------
 * Deformation (Sec. 2: the image pair is warped by the estimate before
 * correlation).
 * ---------------------------------------------------------------------- */

/* Displacement at an arbitrary point: bilinear interpolation of the node
 * field, with the position clamped to the hull of node centres. */
void o_interp(const double* U, int nx, int ny, int step, double x, double y, double* u, double* v) {
  double tx = (x - (step - 1) / 2.0) / step, ty = (y - (step - 1) / 2.0) / step;
  if (tx < 0) tx = 0;
  if (ty < 0) ty = 0;
  if (tx > nx - 1) tx = nx - 1;
  if (ty > ny - 1) ty = ny - 1;
  int bx = (int)floor(tx), by = (int)floor(ty);
  if (bx > nx - 2) bx = nx - 2 < 0 ? 0 : nx - 2;
  if (by > ny - 2) by = ny - 2 < 0 ? 0 : ny - 2;
  double fx = tx - bx, fy = ty - by;
  int bx1 = nx > 1 ? bx + 1 : bx, by1 = ny > 1 ? by + 1 : by;
  for (int c = 0; c < 2; ++c) {
    const double* P = U + (size_t)c * nx * ny;
    double r = (1 - fy) * ((1 - fx) * P[(size_t)by * nx + bx] + fx * P[(size_t)by * nx + bx1]) +
               fy * ((1 - fx) * P[(size_t)by1 * nx + bx] + fx * P[(size_t)by1 * nx + bx1]);
    if (c == 0) *u = r; else *v = r;
  }
}

/* Bilinear sample with zero outside the image. */
double o_bilin(const double* I, int W, int H, double x, double y) {
  double x0 = floor(x), y0 = floor(y);
  double fx = x - x0, fy = y - y0;
  int ix = (int)x0, iy = (int)y0;
  return (1 - fx) * (1 - fy) * dpx(I, W, H, iy, ix) + fx * (1 - fy) * dpx(I, W, H, iy, ix + 1) +
         (1 - fx) * fy * dpx(I, W, H, iy + 1, ix) + fx * fy * dpx(I, W, H, iy + 1, ix + 1);
}

/* Warped value of frame `which` (0 = A, 1 = B) at integer pixel (y, x).
 * mode 0: A' = A, B'(p) = B(p + u(p)).  mode 1 (symmetric, "central"):
 * A'(p) = A(p - u(p)/2), B'(p) = B(p + u(p)/2). */
static double warped(const double* I, int which, int mode, const double* U, int W, int H, int nx,
                     int ny, int step, int y, int x) {
  if (which == 0 && mode == 0) return dpx(I, W, H, y, x);
  double u = 0, v = 0;
  if (U) o_interp(U, nx, ny, step, x, y, &u, &v);
  double s = mode == 1 ? 0.5 : 1.0;
  if (which == 0) s = -s;
  return o_bilin(I, W, H, x + s * u, y + s * v);
}

/* Whole warped image on the pixel grid (for tests). */
void o_warp_image(const double* I, int which, int mode, const double* U, int W, int H, int step,
                  double* out) {
  int nx = W / step, ny = H / step;
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x)
      out[(size_t)y * W + x] = warped(I, which, mode, U, W, H, nx, ny, step, y, x);
}

/* ------------------------------------------------------------------------
 * Correction (Sec. 2: correlation about the estimate, Gaussian sub-pixel
 * fit on the 5-point stencil around the best shift).
 * ---------------------------------------------------------------------- */

/* Three-point Gaussian peak offset on (c-, c0, c+), values floored at 1e-3.
 * Sets *nocurv and returns 0 when the log-parabola does not open downward. */
double o_gauss3(double cm, double c0, double cp, int* nocurv) {
  cm = cm > 1e-3 ? cm : 1e-3;
  c0 = c0 > 1e-3 ? c0 : 1e-3;
  cp = cp > 1e-3 ? cp : 1e-3;
  double lm = log(cm), l0 = log(c0), lp = log(cp);
  double den = 2.0 * (lm - 2.0 * l0 + lp);
  *nocurv = 0;
  if (den >= 0) { *nocurv = 1; return 0.0; }
  return (lm - lp) / den;
}

/* Is (r1, shift1) preferred to (r2, shift2)?  Larger coefficient, then
 * smaller |sx|+|sy|, then smaller sy, then smaller sx. */
static int peak_better(double r1, int sy1, int sx1, double r2, int sy2, int sx2) {
  if (r1 != r2) return r1 > r2;
  int l1 = abs(sx1) + abs(sy1), l2 = abs(sx2) + abs(sy2);
  if (l1 != l2) return l1 < l2;
  if (sy1 != sy2) return sy1 < sy2;
  return sx1 < sx2;
}

/* Pearson correlation coefficient between the (warped) A window of node
 * (a,b) and the warped B window moved by (sy, sx).  *flat is set when the
 * denominator is zero (then 0 is returned). */
static double zncc(const double* A, const double* B, int mode, const double* U, int W, int H,
                   int nx, int ny, int step, int win, int a, int b, int sy, int sx, int* flat) {
  int h = (win - step) / 2, oy = a * step - h, ox = b * step - h;
  double n = (double)win * win, ma = 0, mb = 0;
  for (int i = 0; i < win; ++i)
    for (int j = 0; j < win; ++j) {
      ma += warped(A, 0, mode, U, W, H, nx, ny, step, oy + i, ox + j);
      mb += warped(B, 1, mode, U, W, H, nx, ny, step, oy + i + sy, ox + j + sx);
    }
  ma /= n;
  mb /= n;
  double num = 0, va = 0, vb = 0;
  for (int i = 0; i < win; ++i)
    for (int j = 0; j < win; ++j) {
      double da = warped(A, 0, mode, U, W, H, nx, ny, step, oy + i, ox + j) - ma;
      double db = warped(B, 1, mode, U, W, H, nx, ny, step, oy + i + sy, ox + j + sx) - mb;
      num += da * db;
      va += da * da;
      vb += db * db;
    }
  double den = sqrt(va * vb);
  *flat = !(den > 0);
  return den > 0 ? num / den : 0.0;
}

/* Correlation plane of one window: rho[(sy+r)*(2r+1) + (sx+r)] (for tests). */
void o_corr_plane(const double* A, const double* B, int W, int H, int win, int step, int r, int mode,
                  const double* pred, int a, int b, double* rho) {
  int nx = W / step, ny = H / step, f;
  for (int sy = -r; sy <= r; ++sy)
    for (int sx = -r; sx <= r; ++sx)
      rho[(sy + r) * (2 * r + 1) + sx + r] =
          zncc(A, B, mode, pred, W, H, nx, ny, step, win, a, b, sy, sx, &f);
}

/* Correct the predictor at node (a, b).
 * peak_mode 0: exhaustive argmax over [-r,r]^2, then a 3-point Gaussian fit
 *   per axis about the best shift (none, BORDER, on an axis where the best
 *   shift sits on the search edge);
 * peak_mode 1: the paper's a-priori stencil -- centre fixed at zero shift,
 *   Gaussian fit on the 5 points, offset clamped to [-1, 1].
 * Result = (mean over the window of the interpolated predictor) + best shift
 * + fitted offset: the correlation measures the displacement left after the
 * deformation actually applied to the window's pixels.  *pk receives the
 * coefficient at the chosen shift, *fl the per-vector flags. */
void o_correct_node(const double* A, const double* B, int W, int H, int win, int step, int r,
                    int warp_mode, int peak_mode, const double* pred, int a, int b, double* du,
                    double* dv, double* pk, uint8_t* flo) {
  int nx = W / step, ny = H / step;
  int R = peak_mode == 1 ? 1 : r, S = 2 * R + 1;
  double* rho = (double*)malloc(sizeof(double) * S * S);
  int nflat = 0, nev = 0;
  for (int sy = -R; sy <= R; ++sy)
    for (int sx = -R; sx <= R; ++sx) {
      if (peak_mode == 1 && sx != 0 && sy != 0) { rho[(sy + R) * S + sx + R] = 0; continue; }
      int f;
      rho[(sy + R) * S + sx + R] = zncc(A, B, warp_mode, pred, W, H, nx, ny, step, win, a, b, sy, sx, &f);
      nflat += f;
      nev++;
    }
  uint8_t fl = 0;
  if (nflat == nev) fl |= OF_FLAT;
  int by = 0, bx = 0;
  if (peak_mode == 0) {
    double best = rho[(0 + R) * S + 0 + R];
    for (int sy = -R; sy <= R; ++sy)
      for (int sx = -R; sx <= R; ++sx) {
        double v = rho[(sy + R) * S + sx + R];
        if (peak_better(v, sy, sx, best, by, bx)) { best = v; by = sy; bx = sx; }
      }
  }
  double c0 = rho[(by + R) * S + bx + R];
  double dxs = 0, dys = 0;
  int nc;
  if (peak_mode == 0 && (bx == -R || bx == R)) fl |= OF_BORDER;
  else {
    dxs = o_gauss3(rho[(by + R) * S + bx - 1 + R], c0, rho[(by + R) * S + bx + 1 + R], &nc);
    if (nc) fl |= OF_NOCURV;
  }
  if (peak_mode == 0 && (by == -R || by == R)) fl |= OF_BORDER;
  else {
    dys = o_gauss3(rho[(by - 1 + R) * S + bx + R], c0, rho[(by + 1 + R) * S + bx + R], &nc);
    if (nc) fl |= OF_NOCURV;
  }
  if (peak_mode == 1) {
    dxs = dxs < -1 ? -1 : dxs > 1 ? 1 : dxs;
    dys = dys < -1 ? -1 : dys > 1 ? 1 : dys;
  }
  /* the correction is relative to the deformation applied to the window:
   * add it to the window mean of the interpolated predictor */
  double pu = 0.0, pv = 0.0;
  if (pred) {
    int h = (win - step) / 2;
    for (int i = 0; i < win; ++i)
      for (int j = 0; j < win; ++j) {
        double u, v;
        o_interp(pred, nx, ny, step, b * step - h + j, a * step - h + i, &u, &v);
        pu += u;
        pv += v;
      }
    pu /= (double)win * win;
    pv /= (double)win * win;
  }
  *du = pu + bx + dxs;
  *dv = pv + by + dys;
  *pk = c0;
  *flo = fl;
  free(rho);
}

/* o_correct_node at every node; disp [2][ny][nx], peak (nullable) and flags [ny][nx]. */
void o_correct(const double* A, const double* B, int W, int H, int win, int step, int r,
               int warp_mode, int peak_mode, const double* pred, double* disp, double* peak,
               uint8_t* flags) {
  int nx = W / step, ny = H / step;
  size_t np = (size_t)nx * ny;
#pragma omp parallel for schedule(dynamic)
  for (int a = 0; a < ny; ++a)
    for (int b = 0; b < nx; ++b) {
      size_t i = (size_t)a * nx + b;
      double pk;
      o_correct_node(A, B, W, H, win, step, r, warp_mode, peak_mode, pred, a, b, &disp[i],
                     &disp[np + i], &pk, &flags[i]);
      if (peak) peak[i] = pk;
    }
}

/* ------------------------------------------------------------------------
 * Validation (Sec. 2 and Sec. 3: universal outlier detection, normalised
 * median test with threshold 2 and regulariser 0.1 px; outliers replaced by
 * the median of their non-outlier neighbours).
 * ---------------------------------------------------------------------- */

static int cmp_d(const void* p, const void* q) {
  double a = *(const double*)p, b = *(const double*)q;
  return (a > b) - (a < b);
}

/* median of k values (k >= 1); even k: mean of the two middle values */
static double median_d(double* v, int k) {
  qsort(v, k, sizeof(double), cmp_d);
  return (k & 1) ? v[k / 2] : 0.5 * (v[k / 2 - 1] + v[k / 2]);
}

/* field [2][ny][nx] in/out; flags (nullable) in/out.  A vector whose input
 * flags hold FLAT or BORDER is an outlier and never serves as a neighbour.
 * Detection: over the valid 3x3 neighbours (centre excluded), per component
 * r0 = |u0 - med(u_j)| / (med|u_j - med(u_j)| + eps); outlier when the larger
 * component value exceeds thr.  A vector with no valid neighbour is kept.
 * Replacement, from the detection-pass field: each outlier takes, per
 * component, the median of its non-outlier neighbours; with none it keeps
 * its value and gets UNRESOLVED. */
void o_validate(double* field, uint8_t* flags, int nx, int ny, double thr, double eps) {
  size_t np = (size_t)nx * ny;
  uint8_t* out = (uint8_t*)calloc(np, 1);
  double* orig = (double*)malloc(sizeof(double) * 2 * np);
  memcpy(orig, field, sizeof(double) * 2 * np);
  for (int a = 0; a < ny; ++a)
    for (int b = 0; b < nx; ++b) {
      size_t i = (size_t)a * nx + b;
      if (flags && (flags[i] & (OF_FLAT | OF_BORDER))) { out[i] = 1; continue; }
      double worst = 0;
      int k = 0;
      for (int c = 0; c < 2; ++c) {
        double v[8], dv[8];
        k = 0;
        for (int y = a - 1; y <= a + 1; ++y)
          for (int x = b - 1; x <= b + 1; ++x) {
            if (y < 0 || x < 0 || y >= ny || x >= nx || (y == a && x == b)) continue;
            size_t j = (size_t)y * nx + x;
            if (flags && (flags[j] & (OF_FLAT | OF_BORDER))) continue;
            v[k++] = orig[c * np + j];
          }
        if (k == 0) break;
        double um = median_d(v, k);
        k = 0;
        for (int y = a - 1; y <= a + 1; ++y)
          for (int x = b - 1; x <= b + 1; ++x) {
            if (y < 0 || x < 0 || y >= ny || x >= nx || (y == a && x == b)) continue;
            size_t j = (size_t)y * nx + x;
            if (flags && (flags[j] & (OF_FLAT | OF_BORDER))) continue;
            dv[k++] = fabs(orig[c * np + j] - um);
          }
        double rm = median_d(dv, k);
        double r0 = fabs(orig[c * np + i] - um) / (rm + eps);
        if (r0 > worst) worst = r0;
      }
      if (k > 0 && worst > thr) out[i] = 1;
    }
  for (int a = 0; a < ny; ++a)
    for (int b = 0; b < nx; ++b) {
      size_t i = (size_t)a * nx + b;
      uint8_t fl = flags ? flags[i] : 0;
      if (out[i]) {
        fl |= OF_OUTLIER;
        double v[2][8];
        int k = 0;
        for (int y = a - 1; y <= a + 1; ++y)
          for (int x = b - 1; x <= b + 1; ++x) {
            if (y < 0 || x < 0 || y >= ny || x >= nx || (y == a && x == b)) continue;
            size_t j = (size_t)y * nx + x;
            if (out[j]) continue;
            v[0][k] = orig[j];
            v[1][k] = orig[np + j];
            k++;
          }
        if (k == 0) fl |= OF_UNRESOLVED;
        else {
          field[i] = median_d(v[0], k);
          field[np + i] = median_d(v[1], k);
          fl |= OF_REPLACED;
        }
      }
      if (flags) flags[i] = fl;
    }
  free(out);
  free(orig);
}

/* ------------------------------------------------------------------------
 * Vorticity (Sec. 1 and Sec. 4: displayed and compared with the reference;
 * the scheme is not given).  omega = dv/dx - du/dy on the node grid with
 * spacing h = step: central differences inside, second-order one-sided
 * differences on the first and last node of a line (first order if a line
 * has two nodes, zero if one).
 * ---------------------------------------------------------------------- */

static double deriv(const double* f, int n, int stride, int i, double h) {
  if (n == 1) return 0.0;
  if (n == 2) return (f[stride] - f[0]) / h;
  if (i == 0) return (-3 * f[0] + 4 * f[stride] - f[2 * stride]) / (2 * h);
  if (i == n - 1)
    return (3 * f[(size_t)i * stride] - 4 * f[(size_t)(i - 1) * stride] + f[(size_t)(i - 2) * stride]) / (2 * h);
  return (f[(size_t)(i + 1) * stride] - f[(size_t)(i - 1) * stride]) / (2 * h);
}

void o_vorticity(const double* field, int nx, int ny, int step, double* omega) {
  size_t np = (size_t)nx * ny;
  const double* U = field;
  const double* V = field + np;
  for (int a = 0; a < ny; ++a)
    for (int b = 0; b < nx; ++b) {
      double dvdx = deriv(V + (size_t)a * nx, nx, 1, b, step);
      double dudy = deriv(U + b, ny, nx, a, step);
      omega[(size_t)a * nx + b] = dvdx - dudy;
    }
}

/* ------------------------------------------------------------------------
 * Differentiable windowed SSD (an addition of this implementation, not in
 * the paper): loss per window L_k = sum over the window of (B'(p) - A(p))^2
 * with B'(p) = B(p + u(p)) and u interpolated from the node field U.
 * ---------------------------------------------------------------------- */

void o_ssd_forward(const double* A, const double* B, const double* U, int W, int H, int win, int step,
                   double* loss) {
  int nx = W / step, ny = H / step, h = (win - step) / 2;
#pragma omp parallel for
  for (int a = 0; a < ny; ++a)
    for (int b = 0; b < nx; ++b) {
      double s = 0;
      for (int i = 0; i < win; ++i)
        for (int j = 0; j < win; ++j) {
          int y = a * step - h + i, x = b * step - h + j;
          double u, v;
          o_interp(U, nx, ny, step, x, y, &u, &v);
          double r = o_bilin(B, W, H, x + u, y + v) - dpx(A, W, H, y, x);
          s += r * r;
        }
      loss[(size_t)a * nx + b] = s;
    }
}

/* Gradient of sum_k g_k L_k with respect to U (chain rule through the
 * bilinear sample -- derivative of the floor cell's interpolant -- and the
 * bilinear node interpolation with clamping), and the Gauss-Newton diagonal
 * D = sum_p 2 m(p) (dB'/du)^2 w_n(p)^2 with m(p) = sum of g_k over the
 * windows holding p.  gU, D are [2][ny][nx]; D nullable. */
static int fdiv(int p, int q) { /* floor(p / q), q > 0 */
  return p >= 0 ? p / q : -((-p + q - 1) / q);
}

void o_ssd_grad(const double* A, const double* B, const double* U, const double* g, int W, int H,
                int win, int step, double* gU, double* D) {
  int nx = W / step, ny = H / step, h = (win - step) / 2;
  size_t np = (size_t)nx * ny;
  memset(gU, 0, sizeof(double) * 2 * np);
  if (D) memset(D, 0, sizeof(double) * 2 * np);
  /* every pixel covered by at least one window */
  for (int y = -h; y < ny * step + h; ++y)
    for (int x = -h; x < nx * step + h; ++x) {
      double m = 0;
      int a0 = fdiv(y + h - win + 1, step), a1 = fdiv(y + h, step);
      int b0 = fdiv(x + h - win + 1, step), b1 = fdiv(x + h, step);
      if (a0 < 0) a0 = 0;
      if (b0 < 0) b0 = 0;
      if (a1 > ny - 1) a1 = ny - 1;
      if (b1 > nx - 1) b1 = nx - 1;
      for (int a = a0; a <= a1; ++a)
        for (int b = b0; b <= b1; ++b) {
          int oy = a * step - h, ox = b * step - h;
          if (y >= oy && y < oy + win && x >= ox && x < ox + win) m += g[(size_t)a * nx + b];
        }
      if (m == 0) continue;
      double u, v;
      o_interp(U, nx, ny, step, x, y, &u, &v);
      double qx = x + u, qy = y + v;
      double r = o_bilin(B, W, H, qx, qy) - dpx(A, W, H, y, x);
      double x0 = floor(qx), y0 = floor(qy), fx = qx - x0, fy = qy - y0;
      int ix = (int)x0, iy = (int)y0;
      double p00 = dpx(B, W, H, iy, ix), p01 = dpx(B, W, H, iy, ix + 1);
      double p10 = dpx(B, W, H, iy + 1, ix), p11 = dpx(B, W, H, iy + 1, ix + 1);
      double gx = (1 - fy) * (p01 - p00) + fy * (p11 - p10);
      double gy = (1 - fx) * (p10 - p00) + fx * (p11 - p01);
      /* node weights of u(p), as in o_interp */
      double tx = (x - (step - 1) / 2.0) / step, ty = (y - (step - 1) / 2.0) / step;
      if (tx < 0) tx = 0;
      if (ty < 0) ty = 0;
      if (tx > nx - 1) tx = nx - 1;
      if (ty > ny - 1) ty = ny - 1;
      int bx = (int)floor(tx), by = (int)floor(ty);
      if (bx > nx - 2) bx = nx - 2 < 0 ? 0 : nx - 2;
      if (by > ny - 2) by = ny - 2 < 0 ? 0 : ny - 2;
      double wx = tx - bx, wy = ty - by;
      int bx1 = nx > 1 ? bx + 1 : bx, by1 = ny > 1 ? by + 1 : by;
      int nodes[4] = {by * nx + bx, by * nx + bx1, by1 * nx + bx, by1 * nx + bx1};
      double w[4] = {(1 - wy) * (1 - wx), (1 - wy) * wx, wy * (1 - wx), wy * wx};
      for (int k = 0; k < 4; ++k) {
        gU[nodes[k]] += 2 * m * r * gx * w[k];
        gU[np + nodes[k]] += 2 * m * r * gy * w[k];
        if (D) {
          D[nodes[k]] += 2 * m * gx * gx * w[k] * w[k];
          D[np + nodes[k]] += 2 * m * gy * gy * w[k] * w[k];
        }
      }
    }
}

/* Gradient refinement of U by the windowed SSD (an addition of this
 * implementation, compared with the paper's Gaussian fit): `steps`
 * diagonally preconditioned gradient steps on the total loss
 * L = sum of every window's SSD (upstream gradient 1 for every window):
 *   U <- U - tau * dL/dU / (D + lambda),  lambda = lam_rel * mean(D),
 * D the Gauss-Newton diagonal, mean(D) over both components of the grid.
 * A node component whose D + lambda is not positive is left unchanged.
 * U [2][ny][nx] in/out; hist (nullable) [steps + 1] receives the total loss
 * before each step and after the last. */
void o_ssd_refine(const double* A, const double* B, double* U, int W, int H, int win, int step, int steps,
                  double tau, double lam_rel, double* hist) {
  int nx = W / step, ny = H / step;
  size_t np = (size_t)nx * ny;
  double* loss = (double*)malloc(sizeof(double) * np);
  double* ones = (double*)malloc(sizeof(double) * np);
  double* gU = (double*)malloc(sizeof(double) * 2 * np);
  double* D = (double*)malloc(sizeof(double) * 2 * np);
  for (size_t i = 0; i < np; ++i) ones[i] = 1.0;
  for (int k = 0; k <= steps; ++k) {
    if (hist) {
      o_ssd_forward(A, B, U, W, H, win, step, loss);
      double s = 0;
      for (size_t i = 0; i < np; ++i) s += loss[i];
      hist[k] = s;
    }
    if (k == steps) break;
    o_ssd_grad(A, B, U, ones, W, H, win, step, gU, D);
    double mean = 0;
    for (size_t i = 0; i < 2 * np; ++i) mean += D[i];
    mean /= (double)(2 * np);
    double lam = lam_rel * mean;
    for (size_t i = 0; i < 2 * np; ++i) {
      double den = D[i] + lam;
      if (den > 0) U[i] -= tau * gU[i] / den;
    }
  }
  free(loss);
  free(ones);
  free(gU);
  free(D);
}

/* ------------------------------------------------------------------------
 * Temporal smoothing (Sec. 2: exponential smoothing in time of the
 * validated predictor, constant alpha1, and of the validated final field,
 * constant alpha2).  One frame of one stream: the first frame starts the
 * state (s = x); later frames s = alpha x + (1 - alpha) s.  The field takes
 * the smoothed value.  field, state [2][ny][nx] (np2 values each).
 * ---------------------------------------------------------------------- */
void o_smooth(double* field, double* state, int np2, double alpha, int first) {
  for (int j = 0; j < np2; ++j) {
    double s = first ? field[j] : alpha * field[j] + (1.0 - alpha) * state[j];
    state[j] = s;
    field[j] = s;
  }
}

/* ------------------------------------------------------------------------
 * Pre-processing (Sec. 2: a high-pass filter removes the static background,
 * then contrast-limited adaptive histogram equalisation brightens the
 * image; Sec. 3.1 uses both to match intensities across stitched images).
 * The paper does not specify either filter; these are the readings, in
 * integer arithmetic throughout.
 * ---------------------------------------------------------------------- */

/* High-pass: out = max(0, I - floor(mean of I over the (2r+1)^2 box around
 * the pixel, restricted to the image)).  I, out [H][W]. */
void o_highpass(const int32_t* I, int W, int H, int r, int32_t* out) {
#pragma omp parallel for schedule(static)
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      int64_t s = 0, c = 0;
      for (int v = y - r; v <= y + r; ++v)
        for (int u = x - r; u <= x + r; ++u)
          if (u >= 0 && v >= 0 && u < W && v < H) {
            s += I[(size_t)v * W + u];
            ++c;
          }
      int64_t m = s / c; /* s, c > 0: floor */
      int64_t d = I[(size_t)y * W + x] - m;
      out[(size_t)y * W + x] = (int32_t)(d > 0 ? d : 0);
    }
}

/* Tile boundary j of n tiles over a length L: floor(j L / n). */
static int tile_edge(int j, int L, int n) { return (int)(((int64_t)j * L) / n); }

/* One tile's mapping (contrast-limited equalisation):
 * histogram over nbins (bin = value >> shift); clip every bin at `clip`;
 * the clipped excess is spread evenly: excess / nbins to every bin, then one
 * more to each of the first `rest` bins taken at a stride of
 * max(nbins / rest, 1) from bin 0; lut[b] = round-half-up of
 * cdf(b) * maxval / npix. */
static void clahe_tile_lut(const int32_t* I, int W, int x0, int x1, int y0, int y1, int nbins, int shift,
                           int64_t clip, int maxval, int32_t* lut) {
  int64_t* h = (int64_t*)calloc((size_t)nbins, sizeof(int64_t));
  int64_t npix = (int64_t)(x1 - x0) * (y1 - y0);
  for (int y = y0; y < y1; ++y)
    for (int x = x0; x < x1; ++x) h[I[(size_t)y * W + x] >> shift]++;
  int64_t excess = 0;
  for (int b = 0; b < nbins; ++b)
    if (h[b] > clip) {
      excess += h[b] - clip;
      h[b] = clip;
    }
  int64_t each = excess / nbins, rest = excess - each * nbins;
  for (int b = 0; b < nbins; ++b) h[b] += each;
  if (rest > 0) {
    int64_t stride = nbins / rest;
    if (stride < 1) stride = 1;
    for (int64_t b = 0; b < nbins && rest > 0; b += stride, --rest) h[b]++;
  }
  int64_t cdf = 0;
  for (int b = 0; b < nbins; ++b) {
    cdf += h[b];
    lut[b] = npix > 0 ? (int32_t)((cdf * maxval + npix / 2) / npix) : 0;
  }
  free(h);
}

/* The clip limit of a tile of npix pixels: max(1, floor(clip_factor *
 * npix / nbins)). */
int64_t o_clahe_clip(int64_t npix, int nbins, double clip_factor) {
  double c = floor(clip_factor * (double)npix / (double)nbins);
  return c < 1.0 ? 1 : (int64_t)c;
}

/* CLAHE on a tx x ty grid of tiles (tile j spans [floor(j W/tx),
 * floor((j+1) W/tx)) and likewise in y).  Every tile's mapping is evaluated
 * at the tile centre; a pixel takes the bilinear blend of the mappings of
 * the (up to) four tiles whose centres surround it, clamped at the outer
 * centres; weights are computed in doubled coordinates (centres may be
 * half-integers) and the blend rounds half up, all in integers.
 * bits: meaningful bits of the values (8 for u8); nbins = 2^min(bits, 12). */
void o_clahe(const int32_t* I, int W, int H, int bits, int tx, int ty, double clip_factor, int32_t* out) {
  int lb = bits < 12 ? bits : 12, nbins = 1 << lb, shift = bits - lb, maxval = (1 << bits) - 1;
  int32_t* luts = (int32_t*)malloc(sizeof(int32_t) * (size_t)nbins * tx * ty);
  for (int j = 0; j < ty; ++j)
    for (int i = 0; i < tx; ++i) {
      int x0 = tile_edge(i, W, tx), x1 = tile_edge(i + 1, W, tx);
      int y0 = tile_edge(j, H, ty), y1 = tile_edge(j + 1, H, ty);
      int64_t clip = o_clahe_clip((int64_t)(x1 - x0) * (y1 - y0), nbins, clip_factor);
      clahe_tile_lut(I, W, x0, x1, y0, y1, nbins, shift, clip, maxval, luts + ((size_t)j * tx + i) * nbins);
    }
  for (int y = 0; y < H; ++y)
    for (int x = 0; x < W; ++x) {
      /* doubled coordinates: pixel 2x, tile centre x0 + x1 - 1 */
      int ia = 0, ib = 0, ja = 0, jb = 0;
      int64_t wx = 0, dx = 1, wy = 0, dy = 1;
      int X = 2 * x, Y = 2 * y;
      for (int i = 0; i < tx; ++i)
        if (tile_edge(i, W, tx) + tile_edge(i + 1, W, tx) - 1 <= X) ia = i;
      if (tile_edge(0, W, tx) + tile_edge(1, W, tx) - 1 > X) ia = 0, ib = 0;
      else if (ia == tx - 1) ib = ia;
      else {
        ib = ia + 1;
        int ca = tile_edge(ia, W, tx) + tile_edge(ia + 1, W, tx) - 1;
        int cb = tile_edge(ib, W, tx) + tile_edge(ib + 1, W, tx) - 1;
        wx = X - ca;
        dx = cb - ca;
      }
      for (int j = 0; j < ty; ++j)
        if (tile_edge(j, H, ty) + tile_edge(j + 1, H, ty) - 1 <= Y) ja = j;
      if (tile_edge(0, H, ty) + tile_edge(1, H, ty) - 1 > Y) ja = 0, jb = 0;
      else if (ja == ty - 1) jb = ja;
      else {
        jb = ja + 1;
        int ca = tile_edge(ja, H, ty) + tile_edge(ja + 1, H, ty) - 1;
        int cb = tile_edge(jb, H, ty) + tile_edge(jb + 1, H, ty) - 1;
        wy = Y - ca;
        dy = cb - ca;
      }
      int b = I[(size_t)y * W + x] >> shift;
      int64_t l00 = luts[((size_t)ja * tx + ia) * nbins + b], l01 = luts[((size_t)ja * tx + ib) * nbins + b];
      int64_t l10 = luts[((size_t)jb * tx + ia) * nbins + b], l11 = luts[((size_t)jb * tx + ib) * nbins + b];
      int64_t num = (dy - wy) * ((dx - wx) * l00 + wx * l01) + wy * ((dx - wx) * l10 + wx * l11);
      int64_t den = dx * dy;
      out[(size_t)y * W + x] = (int32_t)((num + den / 2) / den);
    }
  free(luts);
}

/* ------------------------------------------------------------------------
 * Semi-global matching on the node grid (the family of methods the paper's
 * optical-flow engine implements, Sec. 2): the block-SAD cost of every
 * candidate displacement at every node is aggregated along four paths
 * (left to right, right to left, top to bottom, bottom to top) with a small
 * penalty P1 for a change of one pixel in either component between path
 * neighbours and a large penalty P2 for any larger change; the winner
 * minimises (sum over paths, |dx|+|dy|, dy, dx).  Integer throughout.
 * ---------------------------------------------------------------------- */

/* Aggregate a cost volume C[node][k] (nodes row-major on an nx x ny grid, k
 * = (dy+R)(2R+1) + (dx+R) over the (2R+1)^2 candidates) along the four
 * paths; S[node][k] = sum of the four path costs.  Path cost at the first
 * node of a path = C; then
 *   L(p,d) = C(p,d) + min(L(q,d), min_{d' 8-adjacent to d} L(q,d') + P1,
 *                         min_d' L(q,d') + P2) - min_d' L(q,d')
 * with q the previous node on the path. */
void o_sgm_aggregate(const int64_t* C, int nx, int ny, int R, int64_t P1, int64_t P2, int64_t* S) {
  int n1 = 2 * R + 1, nd = n1 * n1;
  size_t np = (size_t)nx * ny;
  memset(S, 0, sizeof(int64_t) * np * nd);
  int64_t* prev = (int64_t*)malloc(sizeof(int64_t) * nd);
  int64_t* cur = (int64_t*)malloc(sizeof(int64_t) * nd);
  /* dir: 0 left->right, 1 right->left, 2 top->bottom, 3 bottom->top */
  for (int dir = 0; dir < 4; ++dir) {
    int nlines = dir < 2 ? ny : nx, len = dir < 2 ? nx : ny;
    for (int line = 0; line < nlines; ++line)
      for (int s = 0; s < len; ++s) {
        int pos = (dir == 1 || dir == 3) ? len - 1 - s : s;
        int a = dir < 2 ? line : pos, b = dir < 2 ? pos : line;
        const int64_t* c = C + ((size_t)a * nx + b) * nd;
        if (s == 0) {
          for (int k = 0; k < nd; ++k) cur[k] = c[k];
        } else {
          int64_t m = prev[0];
          for (int k = 1; k < nd; ++k) if (prev[k] < m) m = prev[k];
          for (int k = 0; k < nd; ++k) {
            int ky = k / n1, kx = k % n1;
            int64_t best = prev[k];
            for (int oy = -1; oy <= 1; ++oy)
              for (int ox = -1; ox <= 1; ++ox) {
                if (!oy && !ox) continue;
                int y2 = ky + oy, x2 = kx + ox;
                if (y2 < 0 || x2 < 0 || y2 >= n1 || x2 >= n1) continue;
                int64_t v = prev[y2 * n1 + x2] + P1;
                if (v < best) best = v;
              }
            if (m + P2 < best) best = m + P2;
            cur[k] = c[k] + best - m;
          }
        }
        int64_t* sp = S + ((size_t)a * nx + b) * nd;
        for (int k = 0; k < nd; ++k) sp[k] += cur[k];
        int64_t* t = prev; prev = cur; cur = t;
      }
  }
  free(prev);
  free(cur);
}

/* One level searched by semi-global matching (no candidate: the search is
 * centred at zero): C from the block SAD of o_sad_level's definition, then
 * o_sgm_aggregate with P1 = p1 block^2 and P2 = p2 block^2, then the winner
 * per node.  d is [2][ny][nx]. */
void o_sgm_level(const int32_t* A, const int32_t* B, int W, int H, int nx, int ny, int step, int block, int R,
                 int p1, int p2, int32_t* d) {
  int off = (step - block) / 2, n1 = 2 * R + 1, nd = n1 * n1;
  size_t np = (size_t)nx * ny;
  int64_t* C = (int64_t*)malloc(sizeof(int64_t) * np * nd);
  int64_t* S = (int64_t*)malloc(sizeof(int64_t) * np * nd);
#pragma omp parallel for schedule(dynamic)
  for (int a = 0; a < ny; ++a)
    for (int b = 0; b < nx; ++b) {
      int oy = a * step + off, ox = b * step + off;
      for (int dy = -R; dy <= R; ++dy)
        for (int dx = -R; dx <= R; ++dx) {
          int64_t s = 0;
          for (int i = 0; i < block; ++i)
            for (int j = 0; j < block; ++j)
              s += llabs((long long)ipx(A, W, H, oy + i, ox + j) - (long long)ipx(B, W, H, oy + i + dy, ox + j + dx));
          C[((size_t)a * nx + b) * nd + (dy + R) * n1 + (dx + R)] = s;
        }
    }
  int64_t bb = (int64_t)block * block;
  o_sgm_aggregate(C, nx, ny, R, (int64_t)p1 * bb, (int64_t)p2 * bb, S);
  for (size_t p = 0; p < np; ++p) {
    int64_t bs = -1;
    int bl = 0, bdy = 0, bdx = 0;
    for (int dy = -R; dy <= R; ++dy)
      for (int dx = -R; dx <= R; ++dx) {
        int64_t s = S[p * nd + (dy + R) * n1 + (dx + R)];
        int l = abs(dx) + abs(dy);
        if (bs < 0 || key_less(s, l, dy, dx, bs, bl, bdy, bdx)) {
          bs = s; bl = l; bdy = dy; bdx = dx;
        }
      }
    d[p] = bdx;
    d[np + p] = bdy;
  }
  free(C);
  free(S);
}
