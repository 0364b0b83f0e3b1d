/*
 * CPU oracle for the thin-disk B-spline self-gravity method — TEST
 * INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library.  It shares no code,
 * header, table or constant with the HIP library.
 *
 * What it computes (all in FP64, no FFT):
 *   - the kernel weights of Eq. (eqnwB) for the order-k tensor B-spline
 *     (Sec. 2.1-2.2, Cases 1-3), by numerical quadrature of their defining
 *     integral: tensor Gauss-Legendre on every spline piece that does not
 *     contain the origin, and a principal-value polar quadrature (Duffy
 *     triangles) on the piece that does (the "removable and integrable"
 *     singularity remark after Eq. (Fx_convolution));
 *   - the discrete convolution of Eq. (eqnF), F_ij = sum C_i'j' w_{i-i',j-j'},
 *     by direct O(M^2 N^2) summation with Neumaier-compensated accumulation;
 *   - the transposed sum (the adjoint of Eq. (eqnF) with respect to C).
 *
 * Spline placement (Sec. 2.2 Cases 1-3 and Sec. 2.3): knots sit at the cell
 * faces x_{i+1/2} = L + i dx.  The spline that multiplies C_i' starts at knot
 * x_{i'-1/2-shift} with shift = floor((k-1)/2), i.e. it is centred on the
 * cell centre x_i' for odd k (k = 3 relabelled so that C_i is centred at x_i,
 * as Eq. (sigmaW) requires) and on the vertex x_{i'+1/2} for k = 2 (Case 2).
 * In the relative variable x~ = x' - x_i the knots are
 *   t_r = (r - m - 1/2 - shift) dx,  r = 0..k,   m = i - i'.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define MAXK 8
#define NQ 6
static const int q_list[NQ] = {4, 6, 8, 12, 20, 32};
static double gl_x[NQ][32], gl_w[NQ][32];
static int gl_ready = 0;

/* Gauss-Legendre nodes and weights on [-1, 1]: Newton iteration on the
 * Legendre polynomial P_q evaluated by its three-term recurrence. */
static void gauss_legendre(int q, double *x, double *w) {
  for (int i = 0; i < q; ++i) {
    long double z = cosl(3.14159265358979323846264338327950288L * (i + 0.75L) / (q + 0.5L));
    long double pp = 1.0L;
    for (int it = 0; it < 100; ++it) {
      long double p1 = 1.0L, p2 = 0.0L;
      for (int j = 1; j <= q; ++j) {
        long double p3 = p2;
        p2 = p1;
        p1 = ((2.0L * j - 1.0L) * z * p2 - (j - 1.0L) * p3) / j;
      }
      pp = q * (z * p1 - p2) / (z * z - 1.0L);
      long double dz = p1 / pp;
      z -= dz;
      if (fabsl(dz) < 1e-19L) break;
    }
    /* recompute the derivative at the converged node */
    long double p1 = 1.0L, p2 = 0.0L;
    for (int j = 1; j <= q; ++j) {
      long double p3 = p2;
      p2 = p1;
      p1 = ((2.0L * j - 1.0L) * z * p2 - (j - 1.0L) * p3) / j;
    }
    pp = q * (z * p1 - p2) / (z * z - 1.0L);
    x[i] = (double)(-z);
    w[i] = (double)(2.0L / ((1.0L - z * z) * pp * pp));
  }
}

static void gl_init(void) {
  if (gl_ready) return;
  for (int a = 0; a < NQ; ++a) gauss_legendre(q_list[a], gl_x[a], gl_w[a]);
  gl_ready = 1;
}

static int q_index(int q) {
  for (int a = 0; a < NQ; ++a)
    if (q_list[a] == q) return a;
  return NQ - 1;
}

/* Value at x of the single order-k B-spline with knots t[0..k], by the
 * Cox-de Boor recursion of Eq. (eqnBk) started from the boxes of
 * Eq. (Bspline1). */
static double bspline(const double *t, int k, double x) {
  double b[MAXK + 1];
  for (int j = 0; j < k; ++j) b[j] = (t[j] <= x && x < t[j + 1]) ? 1.0 : 0.0;
  for (int o = 2; o <= k; ++o)
    for (int j = 0; j + o <= k; ++j) {
      double left = (x - t[j]) / (t[j + o - 1] - t[j]) * b[j];
      double right = (t[j + o] - x) / (t[j + o] - t[j + 1]) * b[j + 1];
      b[j] = left + right;
    }
  return b[0];
}

/* knots of the spline multiplying C_{i'} seen from the cell centre x_i,
 * m = i - i' (see the file header). */
static void knots(int k, int m, double h, double *t) {
  int shift = (k - 1) / 2;
  for (int r = 0; r <= k; ++r) t[r] = ((double)r - (double)m - 0.5 - (double)shift) * h;
}

/* Tensor Gauss-Legendre over one rectangle [xa,xb]x[ya,yb] that does not
 * contain the origin.  The rectangle is halved along its longer side until
 * that side is no longer than the rectangle's distance to the origin, so the
 * kernel's complex singularities stay at least two half-widths away from
 * every quadrature interval (this matters for pieces next to the singular
 * one and for cells with dx != dy); the node count then follows the
 * remaining distance-to-size ratio.  Returns both components (x~/r^3 and
 * y~/r^3 weighted by the spline product). */
static void piece_gl(int k, const double *tx, const double *ty, double xa, double xb, double ya,
                     double yb, double *sx, double *sy) {
  double dxm = (xa > 0) ? xa : ((xb < 0) ? -xb : 0.0);
  double dym = (ya > 0) ? ya : ((yb < 0) ? -yb : 0.0);
  double dist = sqrt(dxm * dxm + dym * dym);
  double w = xb - xa, h = yb - ya;
  double size = fmax(w, h);
  if (size > dist) {
    double ax, ay, bx_, by_;
    if (w >= h) {
      double xm = 0.5 * (xa + xb);
      piece_gl(k, tx, ty, xa, xm, ya, yb, &ax, &ay);
      piece_gl(k, tx, ty, xm, xb, ya, yb, &bx_, &by_);
    } else {
      double ym = 0.5 * (ya + yb);
      piece_gl(k, tx, ty, xa, xb, ya, ym, &ax, &ay);
      piece_gl(k, tx, ty, xa, xb, ym, yb, &bx_, &by_);
    }
    *sx = ax + bx_;
    *sy = ay + by_;
    return;
  }
  double ratio = dist / size;
  int q = ratio < 3 ? 20 : ratio < 20 ? 12 : ratio < 200 ? 8 : ratio < 1000 ? 6 : 4;
  int qi = q_index(q);
  const double *gx = gl_x[qi], *gw = gl_w[qi];
  double cx = 0.5 * (xa + xb), hxp = 0.5 * w;
  double cy = 0.5 * (ya + yb), hyp = 0.5 * h;
  double bx[32], xs[32], by[32], ys[32];
  for (int a = 0; a < q; ++a) {
    xs[a] = cx + hxp * gx[a];
    bx[a] = bspline(tx, k, xs[a]) * gw[a];
    ys[a] = cy + hyp * gx[a];
    by[a] = bspline(ty, k, ys[a]) * gw[a];
  }
  double accx = 0.0, accy = 0.0;
  for (int a = 0; a < q; ++a) {
    double ix = 0.0, iy = 0.0;
    for (int b = 0; b < q; ++b) {
      double r2 = xs[a] * xs[a] + ys[b] * ys[b];
      double inv = by[b] / (r2 * sqrt(r2));
      ix += xs[a] * inv;
      iy += ys[b] * inv;
    }
    accx += bx[a] * ix;
    accy += bx[a] * iy;
  }
  *sx = accx * hxp * hyp;
  *sy = accy * hxp * hyp;
}

/* Principal value over a piece [xa,xb]x[ya,yb] that contains the origin.
 * The piece is cut into the four triangles (O, P, Q) spanned by its edges;
 * a point of a triangle is s*E(u), E(u) = P + u (Q - P), with area element
 * s |P x Q| ds du.  With S the spline product (a polynomial on the piece),
 *   PV = sum_triangles int_0^1 du  c(u) |PxQ| / |E|^3
 *           [ int_0^1 (S(sE) - S(0)) / s ds  +  S(0) ln|E(u)| ],
 * c = E_x (x component) or E_y (y component); the ln(eps) terms cancel
 * because the angular factor integrates to zero over the full circle. */
static void piece_pv(int k, const double *tx, const double *ty, double xa, double xb, double ya,
                     double yb, double *sx, double *sy) {
  const int qu = 32, qs = 20;
  const double *ux = gl_x[q_index(qu)], *uw = gl_w[q_index(qu)];
  const double *sxn = gl_x[q_index(qs)], *swn = gl_w[q_index(qs)];
  double corner[4][2] = {{xb, ya}, {xb, yb}, {xa, yb}, {xa, ya}};
  double S0 = bspline(tx, k, 0.0) * bspline(ty, k, 0.0);
  double accx = 0.0, accy = 0.0;
  for (int e = 0; e < 4; ++e) {
    double Px = corner[e][0], Py = corner[e][1];
    double Qx = corner[(e + 1) % 4][0], Qy = corner[(e + 1) % 4][1];
    double J = fabs(Px * Qy - Py * Qx);
    /* the u-integrand is singular where |E(u)| = 0 off the real axis: split
     * the edge into segments no longer than its distance to the origin */
    double len = sqrt((Qx - Px) * (Qx - Px) + (Qy - Py) * (Qy - Py));
    int nseg = (int)ceil(len / (J / len));
    if (nseg < 1) nseg = 1;
    for (int sg = 0; sg < nseg; ++sg)
    for (int a = 0; a < qu; ++a) {
      double u = (sg + 0.5 * (ux[a] + 1.0)) / nseg, wu = 0.5 * uw[a] / nseg;
      double Ex = Px + u * (Qx - Px), Ey = Py + u * (Qy - Py);
      double E = sqrt(Ex * Ex + Ey * Ey);
      double inner = 0.0;
      for (int b = 0; b < qs; ++b) {
        double s = 0.5 * (sxn[b] + 1.0), ws = 0.5 * swn[b];
        double S = bspline(tx, k, s * Ex) * bspline(ty, k, s * Ey);
        inner += ws * (S - S0) / s;
      }
      inner += S0 * log(E);
      double common = wu * J / (E * E * E) * inner;
      accx += Ex * common;
      accy += Ey * common;
    }
  }
  *sx = accx;
  *sy = accy;
}

/* Both weight components at offset (m, n): w^x_{m,n} (kernel x~/r^3) and
 * w^y_{m,n} (kernel y~/r^3), Eq. (eqnwB), for cell sizes hx, hy. */
static void weight_mn(int k, double hx, double hy, int m, int n, double *wx, double *wy) {
  double tx[MAXK + 1], ty[MAXK + 1];
  knots(k, m, hx, tx);
  knots(k, n, hy, ty);
  double ax = 0.0, ay = 0.0;
  for (int r = 0; r < k; ++r)
    for (int s = 0; s < k; ++s) {
      double xa = tx[r], xb = tx[r + 1], ya = ty[s], yb = ty[s + 1];
      double px, py;
      if (xa < 0 && xb > 0 && ya < 0 && yb > 0)
        piece_pv(k, tx, ty, xa, xb, ya, yb, &px, &py);
      else
        piece_gl(k, tx, ty, xa, xb, ya, yb, &px, &py);
      ax += px;
      ay += py;
    }
  *wx = ax;
  *wy = ay;
}

/* ---------------------------------------------------------------- API -- */

/* Weights at a list of offsets. */
int oracle_weights_at(int k, double hx, double hy, int64_t cnt, const int32_t *ms,
                      const int32_t *ns, double *wx, double *wy) {
  if (k < 1 || k > MAXK) return 1;
  gl_init();
#pragma omp parallel for schedule(dynamic, 64)
  for (int64_t c = 0; c < cnt; ++c) weight_mn(k, hx, hy, ms[c], ns[c], &wx[c], &wy[c]);
  return 0;
}

/* Full tables for an M x N grid: entry (m, n), m in [-(M-1), M-1],
 * n in [-(N-1), N-1], at (n + N - 1) * (2M - 1) + (m + M - 1). */
int oracle_weights_full(int k, int M, int N, double hx, double hy, double *wx, double *wy) {
  if (k < 1 || k > MAXK || M < 1 || N < 1) return 1;
  gl_init();
  const int64_t W = 2 * (int64_t)M - 1;
#pragma omp parallel for schedule(dynamic, 1)
  for (int nn = 0; nn < 2 * N - 1; ++nn)
    for (int mm = 0; mm < W; ++mm)
      weight_mn(k, hx, hy, mm - (M - 1), nn - (N - 1), &wx[nn * W + mm], &wy[nn * W + mm]);
  return 0;
}

/* Neumaier-compensated accumulation */
typedef struct {
  double s, c;
} nsum;
static inline void nadd(nsum *a, double v) {
  double t = a->s + v;
  if (fabs(a->s) >= fabs(v))
    a->c += (a->s - t) + v;
  else
    a->c += (v - t) + a->s;
  a->s = t;
}

/* Eq. (eqnF): F_ij = sum_{i',j'} C_{i'j'} w_{i-i', j-j'} for the listed
 * cells (flat indices j*M + i; all cells when cells == NULL).  C is row-major
 * [N][M] (x fastest); wx, wy are full tables as produced above. */
int oracle_forces(int M, int N, const double *C, const double *wx, const double *wy, int64_t ncells,
                  const int64_t *cells, double *fx, double *fy) {
  const int64_t W = 2 * (int64_t)M - 1;
  int64_t total = cells ? ncells : (int64_t)M * N;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t c = 0; c < total; ++c) {
    int64_t flat = cells ? cells[c] : c;
    int i = (int)(flat % M), j = (int)(flat / M);
    nsum ax = {0, 0}, ay = {0, 0};
    for (int jp = 0; jp < N; ++jp) {
      const double *crow = C + (int64_t)jp * M;
      const double *wxr = wx + (int64_t)(j - jp + N - 1) * W + (i + M - 1);
      const double *wyr = wy + (int64_t)(j - jp + N - 1) * W + (i + M - 1);
      for (int ip = 0; ip < M; ++ip) {
        double cv = crow[ip];
        if (cv == 0.0) continue;
        nadd(&ax, cv * wxr[-ip]);
        nadd(&ay, cv * wyr[-ip]);
      }
    }
    fx[c] = ax.s + ax.c;
    fy[c] = ay.s + ay.c;
  }
  return 0;
}

/* Forces from a sparse coefficient set (positions ip[s], jp[s], values cv[s])
 * at the listed cells, with weights evaluated on the fly: an exact impulse
 * superposition of Eq. (eqnF) that needs no weight table. */
int oracle_forces_sparse(int k, double hx, double hy, int M, int64_t nsrc, const int32_t *ip,
                         const int32_t *jp, const double *cv, int64_t ncells, const int64_t *cells,
                         double *fx, double *fy) {
  if (k < 1 || k > MAXK) return 1;
  gl_init();
#pragma omp parallel for schedule(dynamic, 4)
  for (int64_t c = 0; c < ncells; ++c) {
    int i = (int)(cells[c] % M), j = (int)(cells[c] / M);
    nsum ax = {0, 0}, ay = {0, 0};
    for (int64_t s = 0; s < nsrc; ++s) {
      double wxv, wyv;
      weight_mn(k, hx, hy, i - ip[s], j - jp[s], &wxv, &wyv);
      nadd(&ax, cv[s] * wxv);
      nadd(&ay, cv[s] * wyv);
    }
    fx[c] = ax.s + ax.c;
    fy[c] = ay.s + ay.c;
  }
  return 0;
}

/* Transposed sum: gC_{i'j'} = sum_{ij} wx_{i-i',j-j'} gx_ij + wy_{i-i',j-j'} gy_ij */
int oracle_forces_transpose(int M, int N, const double *gx, const double *gy, const double *wx,
                            const double *wy, double *gc) {
  const int64_t W = 2 * (int64_t)M - 1;
#pragma omp parallel for schedule(dynamic, 16)
  for (int64_t c = 0; c < (int64_t)M * N; ++c) {
    int ip = (int)(c % M), jp = (int)(c / M);
    nsum acc = {0, 0};
    for (int j = 0; j < N; ++j) {
      const double *gxr = gx + (int64_t)j * M, *gyr = gy + (int64_t)j * M;
      const double *wxr = wx + (int64_t)(j - jp + N - 1) * W + (M - 1 - ip);
      const double *wyr = wy + (int64_t)(j - jp + N - 1) * W + (M - 1 - ip);
      for (int i = 0; i < M; ++i) {
        nadd(&acc, gxr[i] * wxr[i]);
        nadd(&acc, gyr[i] * wyr[i]);
      }
    }
    gc[c] = acc.s + acc.c;
  }
  return 0;
}

/* Single B-spline value (exposed for the partition-of-unity and centre-value
 * pins). */
double oracle_bspline(int k, const double *t, double x) { return bspline(t, k, x); }
