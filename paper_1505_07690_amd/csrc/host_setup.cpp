// Host-side FP64 wavelet design of the cake wavelets (Sec. 3.1-3.2): the
// orientation window, its zonal spherical-harmonic coefficients, the Funk
// transform and anti-symmetrisation in coefficient space, the real
// spherical-harmonic recursion shared with the device generator, and the
// steering matrix of the rotated wavelets (Eqs. 17-19).
#include <algorithm>
#include <cmath>

#include "os3d_internal.h"

namespace os3d {

static const double kPi = 3.14159265358979323846;

// Centred cardinal B-spline B^k (Eq. 11: B^k = B^{k-1} * B^0), closed form
// (1/k!) sum_{j=0}^{k+1} (-1)^j C(k+1, j) (x + (k+1)/2 - j)_+^k.
double bspline(int k, double x) {
  double s = 0.0, binom = 1.0;
  for (int j = 0; j <= k + 1; ++j) {
    double t = x + 0.5 * (k + 1) - j;
    double tp = 0.0;
    if (t > 0.0) tp = (k == 0) ? 1.0 : std::pow(t, k);
    s += ((j & 1) ? -binom : binom) * tp;
    binom = binom * (k + 1 - j) / (j + 1);
  }
  double fact = 1.0;
  for (int i = 2; i <= k; ++i) fact *= i;
  return s / fact;
}

// Legendre polynomials P_0..P_L by the three-term recursion.
void legendre(int L, double x, double* P) {
  P[0] = 1.0;
  if (L >= 1) P[1] = x;
  for (int l = 1; l < L; ++l) P[l + 1] = ((2.0 * l + 1.0) * x * P[l] - l * P[l - 1]) / (l + 1.0);
}

// Class-I geodesic icosahedron: planar barycentric subdivision of each of
// the 20 faces into freq^2 triangles, projected to the unit sphere.  The
// base icosahedron has its vertices at the cyclic permutations of
// (0, +-1, +-phi).  Points are generated once each: 12 vertices, freq-1
// interior points per edge, interior points of each face.
std::vector<double> geodesic_icosahedron(int freq) {
  const double ph = 0.5 * (1.0 + std::sqrt(5.0));
  double v[12][3];
  int nv = 0;
  for (double a : {-1.0, 1.0})
    for (double b : {-ph, ph}) {
      double t[3][3] = {{0.0, a, b}, {a, b, 0.0}, {b, 0.0, a}};
      for (auto& q : t) {
        v[nv][0] = q[0];
        v[nv][1] = q[1];
        v[nv][2] = q[2];
        ++nv;
      }
    }
  auto dist2 = [&](int i, int j) {
    double d = 0;
    for (int c = 0; c < 3; ++c) d += (v[i][c] - v[j][c]) * (v[i][c] - v[j][c]);
    return d;
  };
  const double e2 = 4.0;  // squared edge length of this icosahedron
  auto adj = [&](int i, int j) { return i != j && std::fabs(dist2(i, j) - e2) < 1e-9; };
  std::vector<double> out;
  auto emit = [&](double x, double y, double z) {
    double r = std::sqrt(x * x + y * y + z * z);
    out.push_back(x / r);
    out.push_back(y / r);
    out.push_back(z / r);
  };
  for (int i = 0; i < 12; ++i) emit(v[i][0], v[i][1], v[i][2]);
  for (int i = 0; i < 12; ++i)
    for (int j = i + 1; j < 12; ++j)
      if (adj(i, j))
        for (int a = 1; a < freq; ++a) {
          int b = freq - a;
          emit((a * v[i][0] + b * v[j][0]) / freq, (a * v[i][1] + b * v[j][1]) / freq,
               (a * v[i][2] + b * v[j][2]) / freq);
        }
  for (int i = 0; i < 12; ++i)
    for (int j = i + 1; j < 12; ++j)
      for (int k = j + 1; k < 12; ++k)
        if (adj(i, j) && adj(i, k) && adj(j, k))
          for (int a = 1; a < freq; ++a)
            for (int b = 1; a + b < freq; ++b) {
              int c = freq - a - b;
              emit((a * v[i][0] + b * v[j][0] + c * v[k][0]) / freq, (a * v[i][1] + b * v[j][1] + c * v[k][1]) / freq,
                   (a * v[i][2] + b * v[j][2] + c * v[k][2]) / freq);
            }
  return out;
}

// Least-squares fit min ||Y c - values|| with Y[p][l] = sqrt((2l+1)/4pi) P_l(z_p),
// by Householder QR (the pseudo-inverse solution for a full-column-rank Y).
bool zonal_fit(int L, const std::vector<double>& pts, const std::vector<double>& values, std::vector<double>& c) {
  const int m = (int)values.size(), n = L + 1;
  if (m < n) return false;
  std::vector<double> A((size_t)m * n), b(values);
  std::vector<double> P(n);
  for (int p = 0; p < m; ++p) {
    legendre(L, pts[3 * p + 2], P.data());
    for (int l = 0; l < n; ++l) A[(size_t)p * n + l] = std::sqrt((2.0 * l + 1.0) / (4.0 * kPi)) * P[l];
  }
  std::vector<double> diag(n);
  for (int j = 0; j < n; ++j) {
    double norm = 0;
    for (int i = j; i < m; ++i) norm += A[(size_t)i * n + j] * A[(size_t)i * n + j];
    norm = std::sqrt(norm);
    if (norm == 0.0) return false;
    double alpha = A[(size_t)j * n + j] > 0 ? -norm : norm;
    // v = x - alpha e1, stored in column j (rows j..m-1)
    A[(size_t)j * n + j] -= alpha;
    double vnorm2 = 0;
    for (int i = j; i < m; ++i) vnorm2 += A[(size_t)i * n + j] * A[(size_t)i * n + j];
    for (int k = j + 1; k < n; ++k) {
      double s = 0;
      for (int i = j; i < m; ++i) s += A[(size_t)i * n + j] * A[(size_t)i * n + k];
      s = 2.0 * s / vnorm2;
      for (int i = j; i < m; ++i) A[(size_t)i * n + k] -= s * A[(size_t)i * n + j];
    }
    double s = 0;
    for (int i = j; i < m; ++i) s += A[(size_t)i * n + j] * b[i];
    s = 2.0 * s / vnorm2;
    for (int i = j; i < m; ++i) b[i] -= s * A[(size_t)i * n + j];
    diag[j] = alpha;
  }
  c.assign(n, 0.0);
  for (int j = n - 1; j >= 0; --j) {
    double s = b[j];
    for (int k = j + 1; k < n; ++k) s -= A[(size_t)j * n + k] * c[k];
    c[j] = s / diag[j];
  }
  return true;
}

// Cake wavelet (Eq. 14): Funk transform c_l -> 2 pi P_l(0) c_l (Eq. 16) for
// the real line detector, plus anti-symmetrisation c_l -> (1 - (-1)^l) c_l for
// the imaginary edge detector.  Plate variant (Fig. 4): h = A, a_l = c_l.
void cake_coeffs(int L, const double* c, int variant, double* a) {
  std::vector<double> P0(L + 1);
  legendre(L, 0.0, P0.data());
  for (int l = 0; l <= L; ++l) {
    if (variant == OS3D_PLATE)
      a[l] = c[l];
    else
      a[l] = 2.0 * kPi * P0[l] * c[l] + ((l & 1) ? 2.0 : 0.0) * c[l];
  }
}

// Gauss-Legendre nodes (ascending) and weights on [-1, 1]: Newton's method on
// P_n from the asymptotic initial guesses.
static void gauss_legendre(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double z = -std::cos(kPi * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int j = 2; j <= n; ++j) {
        const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int j = 2; j <= n; ++j) {
      const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1.0);
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// c_l = 2 pi int_0^pi A(theta) Y_l0(theta) sin(theta) dtheta, 64 Gauss-Legendre
// nodes on each interval between the knots of B^k(theta / s_theta).
static void quadrature_coeffs(const os3d_wavelet_params& p, std::vector<double>& c) {
  std::vector<double> knots = {0.0, kPi};
  for (int j = 0; j <= p.k + 1; ++j) {
    const double t = p.s_theta * (j - (p.k + 1) / 2.0);
    if (t > 0.0 && t < kPi) knots.push_back(t);
  }
  std::sort(knots.begin(), knots.end());
  knots.erase(std::unique(knots.begin(), knots.end()), knots.end());
  std::vector<double> xg, wg, P(p.L + 1);
  gauss_legendre(64, xg, wg);
  c.assign(p.L + 1, 0.0);
  for (size_t q = 0; q + 1 < knots.size(); ++q) {
    const double a = knots[q], b = knots[q + 1];
    for (int i = 0; i < 64; ++i) {
      const double th = 0.5 * (b - a) * xg[i] + 0.5 * (b + a);
      const double wt = 0.5 * (b - a) * wg[i];
      legendre(p.L, std::cos(th), P.data());
      const double f = bspline(p.k, th / p.s_theta) * std::sin(th) * wt;
      for (int l = 0; l <= p.L; ++l) c[l] += 2.0 * kPi * std::sqrt((2.0 * l + 1.0) / (4.0 * kPi)) * P[l] * f;
    }
  }
}

void wavelet_coeffs(const os3d_wavelet_params& p, std::vector<double>& c, std::vector<double>& a) {
  if (p.coeffs == OS3D_COEFFS_QUADRATURE) {
    quadrature_coeffs(p, c);
  } else {
    std::vector<double> pts = geodesic_icosahedron(15);
    const int np = (int)pts.size() / 3;
    std::vector<double> vals(np);
    for (int i = 0; i < np; ++i) {
      double z = std::max(-1.0, std::min(1.0, pts[3 * i + 2]));
      vals[i] = bspline(p.k, std::acos(z) / p.s_theta);
    }
    zonal_fit(p.L, pts, vals, c);
  }
  a.assign(p.L + 1, 0.0);
  cake_coeffs(p.L, c.data(), p.variant, a.data());
}

ShTables sh_tables(int L) {
  ShTables t;
  t.L = L;
  const int n = L + 1;
  t.qmm.assign(n, 0.0);
  t.alm.assign((size_t)n * n, 0.0);
  t.blm.assign((size_t)n * n, 0.0);
  t.qmm[0] = 1.0 / std::sqrt(4.0 * kPi);
  for (int m = 1; m <= L; ++m) t.qmm[m] = t.qmm[m - 1] * std::sqrt((2.0 * m + 1.0) / (2.0 * m));
  for (int m = 0; m <= L; ++m)
    for (int l = m + 2; l <= L; ++l) {
      t.alm[(size_t)l * n + m] = std::sqrt((4.0 * l * l - 1.0) / ((double)l * l - (double)m * m));
      t.blm[(size_t)l * n + m] =
          std::sqrt(((l - 1.0) * (l - 1.0) - (double)m * m) / (4.0 * (l - 1.0) * (l - 1.0) - 1.0));
    }
  return t;
}

void real_sh(const ShTables& t, const double n[3], double* Y) {
  const int L = t.L, nn = L + 1;
  const double x = n[0], y = n[1], z = n[2];
  double cr = 1.0, ci = 0.0;  // (x + iy)^m
  const double r2 = std::sqrt(2.0);
  for (int m = 0; m <= L; ++m) {
    if (m > 0) {
      double nr = cr * x - ci * y, ni = cr * y + ci * x;
      cr = nr;
      ci = ni;
    }
    double qm2 = 0.0, qm1 = t.qmm[m];
    for (int l = m; l <= L; ++l) {
      double q;
      if (l == m)
        q = t.qmm[m];
      else if (l == m + 1)
        q = std::sqrt(2.0 * m + 3.0) * z * t.qmm[m];
      else
        q = t.alm[(size_t)l * nn + m] * (z * qm1 - t.blm[(size_t)l * nn + m] * qm2);
      if (l > m) {
        qm2 = qm1;
        qm1 = q;
      } else {
        qm1 = q;
      }
      if (m == 0) {
        Y[l * l + l] = q;
      } else {
        Y[l * l + l + m] = r2 * q * cr;
        Y[l * l + l - m] = r2 * q * ci;
      }
    }
  }
}

// Words of orders m0..m1 (one per (l, m), l = m..L).
static int order_words(int L, int m0, int m1) {
  int n = 0;
  for (int m = m0; m <= m1; ++m) n += L + 1 - m;
  return n;
}

int synth_split(int L) {
  int best = L, best_len = order_words(L, 0, L);
  for (int M = 0; M <= L; ++M) {
    const int len = std::max(order_words(L, 0, M), order_words(L, M + 1, L));
    if (len < best_len) {
      best_len = len;
      best = M;
    }
  }
  return best;
}

int synth_pairs(int L) {
  const int M = synth_split(L);
  return std::max(order_words(L, 0, M), order_words(L, M + 1, L));
}

int synth_words(int L) { return 2 * synth_pairs(L); }

int synth_kblocks(int L) { return (synth_words(L) + 15) / 16; }

int synth_sweep_blocks(int ncb) {
  const int sweeps = (ncb + kSynthMaxBlocks - 1) / kSynthMaxBlocks;
  return (ncb + sweeps - 1) / sweeps;
}

int synth_padded_blocks(int ncb) {
  const int per = synth_sweep_blocks(ncb);
  return (ncb + per - 1) / per * per;
}

// The i-th step of a chain over orders m0..m1: (l, m), false past its end.
static bool chain_step(int L, int m0, int m1, int i, int& l, int& m) {
  for (m = m0; m <= m1; ++m) {
    const int n = L + 1 - m;
    if (i < n) {
      l = m + i;
      return true;
    }
    i -= n;
  }
  return false;
}

bool synth_entry(int L, int e, int& l, int& m, bool& sin_part) {
  const int w = e >> 1, i = w >> 1;
  sin_part = (e & 1) == 1;
  const int M = synth_split(L);
  const bool ok = (w & 1) == 0 ? chain_step(L, 0, M, i, l, m) : chain_step(L, M + 1, L, i, l, m);
  return ok && !(m == 0 && sin_part);
}

std::vector<int> synth_word_order(int L) {
  const int M = synth_split(L);
  std::vector<int> lm((size_t)16 * synth_kblocks(L), -1);
  for (int chain = 0; chain < 2; ++chain) {
    int i = 0;
    for (int m = chain == 0 ? 0 : M + 1; m <= (chain == 0 ? M : L); ++m)
      for (int l = m; l <= L; ++l, ++i) lm[(size_t)2 * i + chain] = l * (L + 1) + m;
  }
  return lm;
}

void steering_std(const os3d_wavelet_params& p, const double* orients, int n, const std::vector<double>& a,
                  double* S) {
  const int L = p.L, nk = (L + 1) * (L + 1);
  ShTables t = sh_tables(L);
  std::vector<double> Y(nk);
  for (int i = 0; i < n; ++i) {
    real_sh(t, orients + 3 * i, Y.data());
    for (int l = 0; l <= L; ++l) {
      double w = a[l] * std::sqrt(4.0 * kPi / (2.0 * l + 1.0));
      for (int m = -l; m <= l; ++m) S[(size_t)(l * l + l + m) * n + i] = w * Y[l * l + l + m];
    }
  }
}

void pair_orientations(const double* o, int n, std::vector<int>& partner) {
  partner.assign(n, -1);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      if (j == i) continue;
      double dx = o[3 * i] + o[3 * j], dy = o[3 * i + 1] + o[3 * j + 1], dz = o[3 * i + 2] + o[3 * j + 2];
      if (dx * dx + dy * dy + dz * dz < 1e-18) {
        partner[i] = j;
        break;
      }
    }
}

bool factor235(int64_t n) {
  if (n < 1) return false;
  for (int p : {2, 3, 5})
    while (n % p == 0) n /= p;
  return n == 1;
}

// Radix schedule of a length-n DFT: powers of two in factors of 16 (then 8,
// 4, 2), then 5s and 3s.  The product of the radices is n.
std::vector<int> radix_schedule(int n) {
  std::vector<int> r;
  int m = n;
  int p2 = 0;
  while (m % 2 == 0) {
    m /= 2;
    ++p2;
  }
  while (m % 5 == 0) {
    r.push_back(5);
    m /= 5;
  }
  while (m % 3 == 0) {
    r.push_back(3);
    m /= 3;
  }
  std::vector<int> r2;
  while (p2 >= 4) {
    r2.push_back(16);
    p2 -= 4;
  }
  if (p2 == 3) r2.push_back(8);
  if (p2 == 2) r2.push_back(4);
  if (p2 == 1) r2.push_back(2);
  r2.insert(r2.end(), r.begin(), r.end());
  return r2;
}

}  // namespace os3d
