// Host FP64 construction of the pre-computed quantities of live WDD:
// the kept scan frequencies (Section 6.2), the sampled Hermite-Gauss basis
// (Sections 4 and 5) and the Wiener filter of the pre-computed Wiener filter
// algorithm.  Independent of the device; used by wdd_plan and exported
// through wdd_tables_* for inspection.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <new>
#include <thread>

#include "wdd_internal.h"

namespace {

thread_local std::string g_error;

using cd = std::complex<double>;

// Signed frequency of a 0-based DFT index (indices >= S/2 are negative).
inline int64_t signed_freq(int64_t v, int64_t s) { return (2 * v >= s) ? v - s : v; }

struct Geometry {
  int32_t ny, nx;
  double cy, cx;  // aperture centre in detector pixels
  double r, r2;   // aperture radius and its square
  // Detector rows q_y whose offset u_y = q_y - c_y is inside the aperture, and per row the
  // detector columns [lo, hi] with (q_x - c_x)^2 <= R^2 - u_y^2 (empty rows: lo > hi).
  int64_t qy_lo, qy_hi;
  std::vector<int64_t> row_lo, row_hi;

  void init(int32_t ny_, int32_t nx_, double radius, double cy_, double cx_) {
    ny = ny_; nx = nx_; cy = cy_; cx = cx_; r = radius; r2 = radius * radius;
    qy_lo = std::max<int64_t>(0, (int64_t)std::floor(cy - radius) - 1);
    qy_hi = std::min<int64_t>(ny - 1, (int64_t)std::ceil(cy + radius) + 1);
    if (qy_hi < qy_lo) qy_hi = qy_lo - 1;
    row_lo.assign(std::max<int64_t>(0, qy_hi - qy_lo + 1), 1);
    row_hi.assign(row_lo.size(), 0);
    for (int64_t qy = qy_lo; qy <= qy_hi; ++qy) {
      const double uy = (double)qy - cy;
      const double rem = r2 - uy * uy;
      if (rem < 0) continue;
      // the exact test decides the ends: (q_x - c_x)^2 <= rem
      const double sr = std::sqrt(rem);
      int64_t lo = (int64_t)std::ceil(cx - sr) - 1, hi = (int64_t)std::floor(cx + sr) + 1;
      auto in = [&](int64_t q) { const double u = (double)q - cx; return u * u <= rem; };
      while (lo <= hi && !in(lo)) ++lo;
      while (hi >= lo && !in(hi)) --hi;
      lo = std::max<int64_t>(lo, 0);
      hi = std::min<int64_t>(hi, nx - 1);
      row_lo[qy - qy_lo] = lo;
      row_hi[qy - qy_lo] = hi;
    }
  }

  // True iff some detector pixel q lies in the aperture and in the aperture shifted by -d,
  // i.e. |q - c|^2 <= R^2 and |q - c + d|^2 <= R^2.  Per row the second condition is a
  // convex function of q_x, so the column nearest to c_x - d_x (clamped to the row) decides.
  bool overlaps(double dy, double dx) const {
    for (int64_t qy = qy_lo; qy <= qy_hi; ++qy) {
      const int64_t lo = row_lo[qy - qy_lo], hi = row_hi[qy - qy_lo];
      if (lo > hi) continue;
      const double ry = ((double)qy - cy) + dy;
      const double rem = r2 - ry * ry;
      if (rem < 0) continue;
      int64_t c = (int64_t)std::floor(cx - dx + 0.5);
      c = std::min(std::max(c, lo), hi);
      // both neighbours of the real minimiser are candidates when it falls between columns
      for (int64_t q = std::max(lo, c - 1); q <= std::min(hi, c + 1); ++q) {
        const double rx = ((double)q - cx) + dx;
        if (rx * rx <= rem) return true;
      }
    }
    return false;
  }
};

// W = conj(Y^B) / (|Y^B|^2 + eps_abs), eps_abs = eps_rel max |Y^B|^2 (pre-computed Wiener
// filter algorithm, relative regularisation), in place over t->w which holds Y^B.
void wiener_from_reduced(wdd_tables_s* t) {
  double mx = 0.0;
  for (size_t i = 0; i < t->w.size(); i += 2) mx = std::max(mx, t->w[i] * t->w[i] + t->w[i + 1] * t->w[i + 1]);
  t->eps_abs = t->eps_rel * mx;
  for (size_t i = 0; i < t->w.size(); i += 2) {
    const double re = t->w[i], im = t->w[i + 1];
    const double den = re * re + im * im + t->eps_abs;
    t->w[i] = re / den;
    t->w[i + 1] = -im / den;
  }
}

// Y^B_v[k] = sum_q Y_v[q] exp(+2 pi i (q_y k_y / ny + q_x k_x / nx)) / (ny nx) for the full
// Fourier basis, by separable sums over the pixels of the aperture overlap (FP64).
void fourier_wigner(wdd_tables_s* t, const Geometry& geo) {
  const int32_t ny = t->ny, nx = t->nx, K = ny * nx;
  const int64_t nf = t->n_freq();
  t->w.assign((size_t)nf * K * 2, 0.0);
  std::vector<cd> ey(ny), ex(nx);
  for (int32_t m = 0; m < ny; ++m) ey[m] = std::polar(1.0, 2.0 * M_PI * m / ny);
  for (int32_t m = 0; m < nx; ++m) ex[m] = std::polar(1.0, 2.0 * M_PI * m / nx);
  const double amp = t->amplitude, phi_e = t->defocus, r2 = t->radius * t->radius;
  auto quad_phase = [&](double u) { return cd(std::cos(phi_e * u * u / r2), -std::sin(phi_e * u * u / r2)); };
  const double norm = 1.0 / ((double)ny * nx);
  auto work = [&](int64_t f0, int64_t f1) {
    std::vector<cd> row((size_t)nx), part((size_t)ny * nx);
    for (int64_t f = f0; f < f1; ++f) {
      const int64_t vy = t->freqs[2 * f], vx = t->freqs[2 * f + 1];
      const double dy = (double)signed_freq(vy, t->sy) * ny / (t->sy * t->step);
      const double dx = (double)signed_freq(vx, t->sx) * nx / (t->sx * t->step);
      std::fill(part.begin(), part.end(), cd(0, 0));
      for (int64_t qy = geo.qy_lo; qy <= geo.qy_hi; ++qy) {
        const int64_t lo = geo.row_lo[qy - geo.qy_lo], hi = geo.row_hi[qy - geo.qy_lo];
        if (lo > hi) continue;
        const double uy = (double)qy - geo.cy;
        const double ry = uy + dy;
        const double rem = r2 - ry * ry;
        if (rem < 0) continue;
        const cd rowf = quad_phase(uy) * std::conj(quad_phase(ry));
        bool any = false;
        std::fill(row.begin(), row.end(), cd(0, 0));
        for (int64_t qx = lo; qx <= hi; ++qx) {
          const double ux = (double)qx - geo.cx;
          const double rx = ux + dx;
          if (rx * rx > rem) continue;
          // Y = P(u) conj(P(u + d)); |P| = amp inside both discs
          const cd y = amp * amp * rowf * quad_phase(ux) * std::conj(quad_phase(rx));
          for (int32_t kx = 0; kx < nx; ++kx) row[kx] += y * ex[(qx * kx) % nx];
          any = true;
        }
        if (!any) continue;
        for (int32_t ky = 0; ky < ny; ++ky) {
          const cd e = ey[(qy * ky) % ny];
          cd* dst = &part[(size_t)ky * nx];
          for (int32_t kx = 0; kx < nx; ++kx) dst[kx] += e * row[kx];
        }
      }
      double* out = &t->w[(size_t)f * K * 2];
      for (int32_t k = 0; k < K; ++k) {
        out[2 * k] = part[k].real() * norm;
        out[2 * k + 1] = part[k].imag() * norm;
      }
    }
  };
  unsigned nth = std::max(1u, std::min(64u, std::thread::hardware_concurrency()));
  if (nf < 64) nth = 1;
  std::vector<std::thread> pool;
  const int64_t chunk = (nf + nth - 1) / nth;
  for (unsigned i = 0; i < nth; ++i) {
    const int64_t f0 = i * chunk, f1 = std::min<int64_t>(nf, f0 + chunk);
    if (f0 >= f1) break;
    pool.emplace_back(work, f0, f1);
  }
  for (auto& th : pool) th.join();
}

}  // namespace

namespace wdd {

wdd_status fail(wdd_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  std::vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_error = buf;
  return code;
}

wdd_status build_tables(const wdd_probe* probe, const wdd_scan* scan, const wdd_detector* det,
                        int32_t K, const wdd_options* opts_in, wdd_tables_s* t, bool kept_only) {
  if (!probe || !scan || !det || !t) return fail(WDD_EINVAL, "null argument");
  wdd_options opts;
  wdd_default_options(&opts);
  if (opts_in) opts = *opts_in;
  const double radius = probe->radius_px;
  if (!(radius > 0) || !std::isfinite(radius)) return fail(WDD_EINVAL, "probe radius must be > 0");
  if (!std::isfinite(probe->amplitude) || probe->amplitude == 0.0)
    return fail(WDD_EINVAL, "probe amplitude must be finite and non-zero");
  if (!std::isfinite(probe->defocus_edge_rad)) return fail(WDD_EINVAL, "defocus must be finite");
  if (!std::isfinite(probe->center_y) || !std::isfinite(probe->center_x))
    return fail(WDD_EINVAL, "probe centre must be finite");
  if (scan->sy < 1 || scan->sx < 1 || scan->sy > 4096 || scan->sx > 4096)
    return fail(WDD_EINVAL, "scan size %d x %d outside [1, 4096]", scan->sy, scan->sx);
  if (!(scan->step_px > 0) || !std::isfinite(scan->step_px)) return fail(WDD_EINVAL, "scan step must be > 0");
  if (det->ny < 1 || det->nx < 1 || det->ny > 1024 || det->nx > 1024 || det->nx % 8 != 0)
    return fail(WDD_EINVAL, "detector %d x %d: need 1 <= ny, nx <= 1024 and nx a multiple of 8", det->ny, det->nx);
  if (det->dtype != WDD_U16 && det->dtype != WDD_F32) return fail(WDD_EINVAL, "unknown frame dtype %d", det->dtype);
  const bool fourier = opts.basis == WDD_BASIS_FOURIER;
  if (opts.basis != WDD_BASIS_HERMITE_GAUSS && !fourier) return fail(WDD_EINVAL, "unknown basis %d", opts.basis);
  auto pow2 = [](int32_t n) { return n > 0 && (n & (n - 1)) == 0; };
  if (fourier) {
    if (!pow2(det->ny) || !pow2(det->nx) || det->ny < 8 || det->nx < 8 || det->ny > 64 || det->nx > 64)
      return fail(WDD_EINVAL, "the Fourier basis needs ny, nx powers of two in [8, 64] (got %d x %d)", det->ny,
                  det->nx);
    if (K != det->ny * det->nx) return fail(WDD_EINVAL, "the Fourier basis has K = ny nx = %d (got %d)",
                                            det->ny * det->nx, K);
  } else if (K < 1 || K > 256) {
    return fail(WDD_EINVAL, "K = %d outside [1, 256]", K);
  }
  if (!(opts.eps_rel > 0) || !std::isfinite(opts.eps_rel)) return fail(WDD_EINVAL, "eps_rel must be > 0");
  if (!std::isfinite(opts.sigma_px)) return fail(WDD_EINVAL, "sigma must be finite");

  int32_t L = 1;
  while (L * L < K) ++L;
  if (fourier) L = 0;
  t->sy = scan->sy; t->sx = scan->sx; t->ny = det->ny; t->nx = det->nx; t->k = K; t->l = L;
  t->step = scan->step_px; t->radius = radius; t->amplitude = probe->amplitude;
  t->cy = probe->center_y; t->cx = probe->center_x;
  t->defocus = probe->defocus_edge_rad; t->eps_rel = opts.eps_rel;
  t->sigma = fourier ? 0.0 : (opts.sigma_px > 0 ? opts.sigma_px : radius / std::sqrt(2.0 * L - 1.0));
  t->basis = opts.basis;

  try {
    // --- kept frequencies -------------------------------------------------
    Geometry geo;
    geo.init(t->ny, t->nx, radius, t->cy, t->cx);
    const double reach = 2.0 * radius + 2.0;
    t->freqs.clear();
    for (int64_t vy = 0; vy < t->sy; ++vy) {
      const double dy = (double)signed_freq(vy, t->sy) * t->ny / (t->sy * t->step);
      if (std::fabs(dy) > reach) continue;
      for (int64_t vx = 0; vx < t->sx; ++vx) {
        const double dx = (double)signed_freq(vx, t->sx) * t->nx / (t->sx * t->step);
        if (std::fabs(dx) > reach) continue;
        if (geo.overlaps(dy, dx)) {
          t->freqs.push_back((int32_t)vy);
          t->freqs.push_back((int32_t)vx);
        }
      }
    }

    if (t->freqs.empty())
      return fail(WDD_EINVAL, "the aperture (radius %g at (%g, %g)) covers no pixel of the %d x %d detector", radius,
                  t->cy, t->cx, t->ny, t->nx);
    if (kept_only) return WDD_OK;

    if (fourier) {
      fourier_wigner(t, geo);
      wiener_from_reduced(t);
      return WDD_OK;
    }

    // --- Hermite-Gauss basis ---------------------------------------------
    auto sample = [&](int32_t n, double c, std::vector<double>& psi) {
      psi.assign((size_t)n * L, 0.0);
      for (int32_t i = 0; i < n; ++i) {
        const double x = ((double)i - c) / t->sigma;
        double pm = 0.0, p = std::pow(M_PI, -0.25) * std::exp(-0.5 * x * x);
        psi[(size_t)i * L] = p;
        for (int32_t m = 0; m + 1 < L; ++m) {
          const double next = std::sqrt(2.0 / (m + 1)) * x * p - std::sqrt((double)m / (m + 1)) * pm;
          pm = p;
          p = next;
          psi[(size_t)i * L + m + 1] = p;
        }
      }
      for (int32_t m = 0; m < L; ++m) {
        double s = 0.0;
        for (int32_t i = 0; i < n; ++i) s += psi[(size_t)i * L + m] * psi[(size_t)i * L + m];
        const double inv = s > 0 ? 1.0 / std::sqrt(s) : 0.0;
        for (int32_t i = 0; i < n; ++i) psi[(size_t)i * L + m] *= inv;
      }
    };
    sample(t->ny, t->cy, t->psi_y);
    sample(t->nx, t->cx, t->psi_x);

    std::vector<std::pair<int32_t, int32_t>> pr;
    for (int32_t a = 0; a < L; ++a)
      for (int32_t b = 0; b < L; ++b) pr.emplace_back(a, b);
    std::sort(pr.begin(), pr.end(), [](const std::pair<int32_t, int32_t>& p, const std::pair<int32_t, int32_t>& q) {
      const int32_t mp = std::max(p.first, p.second), mq = std::max(q.first, q.second);
      if (mp != mq) return mp < mq;
      const int32_t sp = p.first + p.second, sq = q.first + q.second;
      if (sp != sq) return sp < sq;
      return p.first < q.first;
    });
    t->pairs.resize((size_t)2 * K);
    for (int32_t k = 0; k < K; ++k) {
      t->pairs[2 * k] = pr[k].first;
      t->pairs[2 * k + 1] = pr[k].second;
    }

    // --- reduced probe Wigner functions Y^B_v = Phi^T vec(Y_v) -------------
    const int64_t nf = t->n_freq();
    t->w.assign((size_t)nf * K * 2, 0.0);
    const double amp = t->amplitude, phi_e = t->defocus, r2 = radius * radius;
    const int64_t rows = std::max<int64_t>(0, geo.qy_hi - geo.qy_lo + 1);
    // The aperture's quadratic phase is separable in (u_y, u_x).
    auto quad_phase = [&](double u) { return cd(std::cos(phi_e * u * u / r2), -std::sin(phi_e * u * u / r2)); };
    std::vector<cd> p0y(rows), p0x(t->nx);
    for (int64_t qy = geo.qy_lo; qy <= geo.qy_hi; ++qy) p0y[qy - geo.qy_lo] = quad_phase((double)qy - geo.cy);
    for (int32_t qx = 0; qx < t->nx; ++qx) p0x[qx] = quad_phase((double)qx - geo.cx);

    auto work = [&](int64_t f0, int64_t f1) {
      std::vector<cd> py(rows), px(t->nx), tr(L), g((size_t)L * L);
      for (int64_t f = f0; f < f1; ++f) {
        const int64_t vy = t->freqs[2 * f], vx = t->freqs[2 * f + 1];
        const double dy = (double)signed_freq(vy, t->sy) * t->ny / (t->sy * t->step);
        const double dx = (double)signed_freq(vx, t->sx) * t->nx / (t->sx * t->step);
        for (int64_t qy = geo.qy_lo; qy <= geo.qy_hi; ++qy) py[qy - geo.qy_lo] = quad_phase(((double)qy - geo.cy) + dy);
        for (int32_t qx = 0; qx < t->nx; ++qx) px[qx] = quad_phase(((double)qx - geo.cx) + dx);
        std::fill(g.begin(), g.end(), cd(0, 0));
        for (int64_t qy = geo.qy_lo; qy <= geo.qy_hi; ++qy) {
          const int64_t lo = geo.row_lo[qy - geo.qy_lo], hi = geo.row_hi[qy - geo.qy_lo];
          if (lo > hi) continue;
          const double ry = ((double)qy - geo.cy) + dy;
          const double rem = r2 - ry * ry;
          if (rem < 0) continue;
          // columns of this row inside the shifted disc: (q_x - c_x + d_x)^2 <= rem
          const double sr = std::sqrt(rem);
          const int64_t a = std::max<int64_t>(lo, (int64_t)std::ceil(geo.cx - dx - sr) - 1);
          const int64_t b = std::min<int64_t>(hi, (int64_t)std::floor(geo.cx - dx + sr) + 1);
          std::fill(tr.begin(), tr.end(), cd(0, 0));
          bool any = false;
          const cd rowf = p0y[qy - geo.qy_lo] * std::conj(py[qy - geo.qy_lo]);
          for (int64_t qx = a; qx <= b; ++qx) {
            const double rx = ((double)qx - geo.cx) + dx;
            if (rx * rx > rem) continue;
            // Y = P(u) conj(P(u + d)); |P| = amp inside both discs
            const cd y = amp * amp * rowf * p0x[qx] * std::conj(px[qx]);
            const double* ps = &t->psi_x[(size_t)qx * L];
            for (int32_t m = 0; m < L; ++m) tr[m] += y * ps[m];
            any = true;
          }
          if (!any) continue;
          const double* ps = &t->psi_y[(size_t)qy * L];
          for (int32_t a2 = 0; a2 < L; ++a2)
            for (int32_t m = 0; m < L; ++m) g[(size_t)a2 * L + m] += ps[a2] * tr[m];
        }
        double* out = &t->w[(size_t)f * K * 2];
        for (int32_t k = 0; k < K; ++k) {
          const cd v = g[(size_t)t->pairs[2 * k] * L + t->pairs[2 * k + 1]];
          out[2 * k] = v.real();
          out[2 * k + 1] = v.imag();
        }
      }
    };
    unsigned nth = std::max(1u, std::min(64u, std::thread::hardware_concurrency()));
    if (nf < 64) nth = 1;
    std::vector<std::thread> pool;
    const int64_t chunk = (nf + nth - 1) / nth;
    for (unsigned i = 0; i < nth; ++i) {
      const int64_t f0 = i * chunk, f1 = std::min<int64_t>(nf, f0 + chunk);
      if (f0 >= f1) break;
      pool.emplace_back(work, f0, f1);
    }
    for (auto& th : pool) th.join();

    wiener_from_reduced(t);
  } catch (const std::bad_alloc&) {
    return fail(WDD_ENOMEM, "host tables do not fit in memory");
  } catch (const std::system_error&) {
    return fail(WDD_ENOMEM, "could not start table worker threads");
  }
  return WDD_OK;
}

}  // namespace wdd

extern "C" {

const char* wdd_last_error(void) { return g_error.c_str(); }

wdd_status wdd_default_options(wdd_options* opts) {
  if (!opts) return wdd::fail(WDD_EINVAL, "null options");
  opts->eps_rel = 0.01;
  opts->sigma_px = 0.0;
  opts->precision = WDD_FP32;
  opts->max_batch = 256;
  opts->order = WDD_ORDER_SPECTRUM;
  opts->basis = WDD_BASIS_HERMITE_GAUSS;
  opts->pipeline = 0;
  return WDD_OK;
}

wdd_status wdd_tables_build(const wdd_probe* probe, const wdd_scan* scan, const wdd_detector* det, int32_t K,
                            const wdd_options* opts, wdd_tables_t* out) {
  if (!out) return wdd::fail(WDD_EINVAL, "null output handle");
  *out = nullptr;
  wdd_tables_s* t = new (std::nothrow) wdd_tables_s();
  if (!t) return wdd::fail(WDD_ENOMEM, "out of host memory");
  const wdd_status st = wdd::build_tables(probe, scan, det, K, opts, t);
  if (st != WDD_OK) {
    delete t;
    return st;
  }
  *out = t;
  return WDD_OK;
}

wdd_status wdd_tables_info(wdd_tables_t t, wdd_plan_info* info) {
  if (!t || !info) return wdd::fail(WDD_EINVAL, "null argument");
  *info = wdd_plan_info{};
  info->n_freq = t->n_freq();
  info->k = t->k;
  info->l = t->l;
  info->sigma_px = t->sigma;
  info->eps_abs = t->eps_abs;
  return WDD_OK;
}

wdd_status wdd_tables_export(wdd_tables_t t, int32_t* freqs, double* psi_y, double* psi_x, int32_t* pairs,
                             double* w) {
  if (!t) return wdd::fail(WDD_EINVAL, "null tables");
  if (freqs) std::copy(t->freqs.begin(), t->freqs.end(), freqs);
  if (psi_y) std::copy(t->psi_y.begin(), t->psi_y.end(), psi_y);
  if (psi_x) std::copy(t->psi_x.begin(), t->psi_x.end(), psi_x);
  if (pairs) std::copy(t->pairs.begin(), t->pairs.end(), pairs);
  if (w) std::copy(t->w.begin(), t->w.end(), w);
  return WDD_OK;
}

wdd_status wdd_tables_free(wdd_tables_t t) {
  delete t;
  return WDD_OK;
}

}  // extern "C"
