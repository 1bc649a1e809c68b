// Image-domain screens Phi_qc(l, m) of the Mueller kernels, host float64.
//
// Sec. 3.2: Mueller matrices from the Jones matrices of a baseline's two antennas,
// M = J_a (x) conj(J_b) (identical antennas: J_b = J_a) in correlation order XX, XY, YX, YY (Eq. 3); Stokes form
// M^S = S M S^-1 with S from Eq. 4 (U = (XY + YX)/2 by default, the printed
// U = i (XY + YX)/2 on request).  Gridding screens are (M'^S)^-1 S, where M' has
// its diagonal regularised by Eq. 6 (Sec. 3.3); degridding screens are
// (S^-1 M^S)^H, whose conjugate carries the Stokes sky to observed correlations.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <complex>
#include <string>
#include <thread>
#include <vector>

#include "common.hpp"

namespace pg {
namespace {

using cd = std::complex<double>;

// Runs fn(begin, end) over [0, n) split across host threads (per-pixel work is independent).
template <class F>
void parallel_for(size_t n, F fn) {
  const size_t hw = std::max(1u, std::thread::hardware_concurrency());
  const size_t nt = std::min<size_t>({hw, 16, std::max<size_t>(1, n / 4096)});
  if (nt <= 1) {
    fn(size_t{0}, n);
    return;
  }
  std::vector<std::thread> th;
  const size_t step = (n + nt - 1) / nt;
  for (size_t t = 0; t < nt; ++t) {
    const size_t b = t * step, e = std::min(n, b + step);
    if (b < e) th.emplace_back(fn, b, e);
  }
  for (auto& x : th) x.join();
}

struct M4 {
  cd a[4][4];
};

M4 mul(const M4& x, const M4& y) {
  M4 r;
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      cd s = 0.0;
      for (int k = 0; k < 4; ++k) s += x.a[i][k] * y.a[k][j];
      r.a[i][j] = s;
    }
  return r;
}

// Gauss-Jordan inverse with partial pivoting; false if singular.
bool inverse(const M4& m, M4& out) {
  cd w[4][8];
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) {
      w[i][j] = m.a[i][j];
      w[i][j + 4] = (i == j) ? 1.0 : 0.0;
    }
  for (int col = 0; col < 4; ++col) {
    int piv = col;
    for (int r = col + 1; r < 4; ++r)
      if (std::abs(w[r][col]) > std::abs(w[piv][col])) piv = r;
    if (std::abs(w[piv][col]) == 0.0) return false;
    if (piv != col)
      for (int j = 0; j < 8; ++j) std::swap(w[piv][j], w[col][j]);
    cd inv = 1.0 / w[col][col];
    for (int j = 0; j < 8; ++j) w[col][j] *= inv;
    for (int r = 0; r < 4; ++r) {
      if (r == col) continue;
      cd f = w[r][col];
      if (f == 0.0) continue;
      for (int j = 0; j < 8; ++j) w[r][j] -= f * w[col][j];
    }
  }
  for (int i = 0; i < 4; ++i)
    for (int j = 0; j < 4; ++j) out.a[i][j] = w[i][j + 4];
  return true;
}

M4 stokes(int convention) {
  M4 s;
  for (auto& row : s.a)
    for (auto& v : row) v = 0.0;
  s.a[0][0] = 0.5;
  s.a[0][3] = 0.5;
  s.a[1][0] = 0.5;
  s.a[1][3] = -0.5;
  cd u = convention == PG_STOKES_PAPER ? cd(0.0, 0.5) : cd(0.5, 0.0);
  s.a[2][1] = u;
  s.a[2][2] = u;
  s.a[3][1] = cd(0.0, -0.5);
  s.a[3][2] = cd(0.0, 0.5);
  return s;
}

}  // namespace

bool build_screens(int npol, int kind, const double* jones, const double* jones_b, int mk, double eps, int convention,
                   std::vector<double>& phi, std::string& err) {
  const size_t npix = static_cast<size_t>(mk) * mk;
  if (npol == 1) {
    if (jones || jones_b) {
      err = "npol = 1 (Stokes I only) takes no Jones field";
      return false;
    }
    phi.assign(2 * npix, 0.0);
    for (size_t i = 0; i < npix; ++i) phi[2 * i] = 1.0;
    return true;
  }
  const M4 s = stokes(convention);
  M4 sinv;
  if (!inverse(s, sinv)) {
    err = "Stokes matrix is singular";
    return false;
  }
  // M^S at every lattice sample.
  std::vector<M4> ms(npix);
  parallel_for(npix, [&](size_t px0, size_t px1) {
  for (size_t px = px0; px < px1; ++px) {
    // the baseline's two antennas: J_a from `jones`, J_b from `jones_b` (identical antennas when NULL)
    cd ja[2][2], jb[2][2];
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        const size_t o = 2 * ((static_cast<size_t>(a) * 2 + b) * npix + px);
        ja[a][b] = jones ? cd(jones[o], jones[o + 1]) : cd((a == b) ? 1.0 : 0.0);
        jb[a][b] = jones_b ? cd(jones_b[o], jones_b[o + 1]) : ja[a][b];
      }
    M4 m;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        for (int c = 0; c < 2; ++c)
          for (int d = 0; d < 2; ++d) m.a[2 * a + b][2 * c + d] = ja[a][c] * std::conj(jb[b][d]);
    ms[px] = mul(mul(s, m), sinv);
  }
  });
  phi.assign(2 * 16 * npix, 0.0);
  if (kind == PG_KIND_GRID) {
    double beta[4];
    for (int p = 0; p < 4; ++p) {
      double mx = 0.0;
      for (size_t px = 0; px < npix; ++px) mx = std::max(mx, std::abs(ms[px].a[p][p]));
      beta[p] = (eps / 2.0) * mx * (eps / 2.0) * mx;
    }
    std::atomic<bool> singular{false};
    parallel_for(npix, [&](size_t px0, size_t px1) {
    for (size_t px = px0; px < px1; ++px) {
      M4 reg = ms[px];
      for (int p = 0; p < 4; ++p) {  // Eq. 6 on a copy of the diagonal
        cd b = reg.a[p][p];
        if (std::abs(b) == 0.0) b = 1e-150;
        double mag2 = std::norm(b);
        reg.a[p][p] = b * (1.0 + beta[p] / mag2);
      }
      M4 inv;
      if (!inverse(reg, inv)) {
        singular = true;
        continue;
      }
      M4 f = mul(inv, s);
      for (int q = 0; q < 4; ++q)
        for (int c = 0; c < 4; ++c) {
          size_t o = 2 * ((static_cast<size_t>(q) * 4 + c) * npix + px);
          phi[o] = f.a[q][c].real();
          phi[o + 1] = f.a[q][c].imag();
        }
    }
    });
    if (singular) {
      err = "regularised Stokes Mueller matrix is singular at a lattice sample";
      return false;
    }
  } else {
    parallel_for(npix, [&](size_t px0, size_t px1) {
    for (size_t px = px0; px < px1; ++px) {
      M4 a = mul(sinv, ms[px]);
      for (int q = 0; q < 4; ++q)
        for (int c = 0; c < 4; ++c) {
          cd v = std::conj(a.a[c][q]);
          size_t o = 2 * ((static_cast<size_t>(q) * 4 + c) * npix + px);
          phi[o] = v.real();
          phi[o + 1] = v.imag();
        }
    }
    });
  }
  return true;
}

}  // namespace pg
