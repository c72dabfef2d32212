// Host-side assembly of the transfer weights (Section 3 of Stokes et al.,
// arXiv 2504.15814: per expansion cell, a Taylor polynomial is fitted through
// the values of a stencil of cell centres and evaluated at the target
// centres; Appendix C: central stencils inside the face, shifted toward the
// face interior near its edges and vertices).
//
// The fits are solved once per class of expansion cell, in long double, with
// a Householder QR of the stencil matrix, and rounded to float64 / float32
// weight blocks.  A block holds the weights of all R targets that share one
// expansion anchor column, over the union of their source cells.
#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <tuple>

#include "ft_internal.h"

namespace ft {
namespace {

using Vec3 = std::array<long double, 3>;
using Cell = std::tuple<int, int, int>;  // (n, b, c) in the reference frame
using Row = std::map<Cell, long double>;

// Monomial exponents with 1 <= |alpha| <= degree (the constant is pinned), in
// `dim` variables (the third exponent is zero in two dimensions).
std::vector<std::array<int, 3>> exponents(int degree, int dim) {
  std::vector<std::array<int, 3>> out;
  for (int t = 1; t <= degree; ++t)
    for (int e0 = t; e0 >= 0; --e0) {
      if (dim == 2) {
        out.push_back({e0, t - e0, 0});
        continue;
      }
      for (int e1 = t - e0; e1 >= 0; --e1) out.push_back({e0, e1, t - e0 - e1});
    }
  return out;
}

long double monomial(const Vec3& d, const std::array<int, 3>& e) {
  long double v = 1.0L;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < e[i]; ++j) v *= d[i];
  return v;
}

// Least squares with the constant pinned to the centre value: returns one
// weight row over `offs` per target.  Householder QR of the (s-1) x n matrix
// of monomials at the non-centre offsets; X = R^{-1} Q^T is the map from
// (values - centre value) to the monomial coefficients.
bool pinned_fit(const std::vector<Vec3>& offs, int centre, int degree, int dim,
                const std::vector<Vec3>& targets, std::vector<std::vector<long double>>* W,
                std::string* err) {
  const auto ex = exponents(degree, dim);
  const int n = (int)ex.size();
  std::vector<int> others;
  for (int q = 0; q < (int)offs.size(); ++q)
    if (q != centre) others.push_back(q);
  const int m = (int)others.size();
  if (m < n) {
    *err = "stencil smaller than the number of derivatives";
    return false;
  }
  std::vector<std::vector<long double>> A(m, std::vector<long double>(n));
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) A[i][j] = monomial(offs[others[i]], ex[j]);
  // B accumulates Q^T (m x m).
  std::vector<std::vector<long double>> B(m, std::vector<long double>(m, 0.0L));
  for (int i = 0; i < m; ++i) B[i][i] = 1.0L;
  long double scale = 0.0L;
  for (int i = 0; i < m; ++i)
    for (int j = 0; j < n; ++j) scale = std::max(scale, std::fabs(A[i][j]));
  for (int j = 0; j < n; ++j) {
    long double norm = 0.0L;
    for (int i = j; i < m; ++i) norm += A[i][j] * A[i][j];
    norm = std::sqrt(norm);
    if (norm <= 1e-12L * scale) {
      *err = "stencil does not determine all derivatives (rank deficient)";
      return false;
    }
    const long double alpha = A[j][j] > 0 ? -norm : norm;
    std::vector<long double> v(m, 0.0L);
    v[j] = A[j][j] - alpha;
    for (int i = j + 1; i < m; ++i) v[i] = A[i][j];
    long double vv = 0.0L;
    for (int i = j; i < m; ++i) vv += v[i] * v[i];
    if (vv == 0.0L) continue;
    auto reflect = [&](std::vector<std::vector<long double>>& M, int c0, int ncols) {
      for (int c = c0; c < ncols; ++c) {
        long double dot = 0.0L;
        for (int i = j; i < m; ++i) dot += v[i] * M[i][c];
        const long double f = 2.0L * dot / vv;
        for (int i = j; i < m; ++i) M[i][c] -= f * v[i];
      }
    };
    reflect(A, j, n);
    reflect(B, 0, m);
  }
  // X = R^{-1} (Q^T)[0:n, :], by back substitution column by column.
  std::vector<std::vector<long double>> X(n, std::vector<long double>(m, 0.0L));
  for (int c = 0; c < m; ++c)
    for (int i = n - 1; i >= 0; --i) {
      long double acc = B[i][c];
      for (int j = i + 1; j < n; ++j) acc -= A[i][j] * X[j][c];
      X[i][c] = acc / A[i][i];
    }
  W->assign(targets.size(), std::vector<long double>(offs.size(), 0.0L));
  for (size_t t = 0; t < targets.size(); ++t) {
    std::vector<long double> mono(n);
    for (int j = 0; j < n; ++j) mono[j] = monomial(targets[t], ex[j]);
    long double sum = 0.0L;
    for (int c = 0; c < m; ++c) {
      long double w = 0.0L;
      for (int j = 0; j < n; ++j) w += mono[j] * X[j][c];
      (*W)[t][others[c]] = w;
      sum += w;
    }
    (*W)[t][centre] = 1.0L - sum;
  }
  return true;
}

// Stencil along one axis: box of three around the centre clamped into
// [lo+1, hi-1], plus (degree 3) the points two away from the box centre.
void axis_box(int centre, int lo, int hi, int* box_mid) {
  *box_mid = std::min(std::max(centre, lo + 1), hi - 1);
}

// In two dimensions the third coordinate is 0 and the box is 3 x 3.
std::vector<Cell> taylor_stencil(int degree, int dim, Cell centre, const int lo[3],
                                 const int hi[3]) {
  int mid[3];
  const int cc[3] = {std::get<0>(centre), std::get<1>(centre), std::get<2>(centre)};
  for (int i = 0; i < dim; ++i) axis_box(cc[i], lo[i], hi[i], &mid[i]);
  if (dim == 2) mid[2] = 0;
  const int r2 = dim == 3 ? 1 : 0;
  std::vector<Cell> pts;
  for (int d0 = -1; d0 <= 1; ++d0)
    for (int d1 = -1; d1 <= 1; ++d1)
      for (int d2 = -r2; d2 <= r2; ++d2) pts.emplace_back(mid[0] + d0, mid[1] + d1, mid[2] + d2);
  if (degree >= 3) {
    for (int ax = 0; ax < dim; ++ax)
      for (int st = -2; st <= 2; st += 4) {
        int q[3] = {mid[0], mid[1], mid[2]};
        q[ax] += st;
        if (q[ax] >= lo[ax] && q[ax] <= hi[ax]) pts.emplace_back(q[0], q[1], q[2]);
      }
  }
  return pts;
}

// Taylor rows about `centre` (reference cells, spacing `unit` per index)
// evaluated at the given target offsets (in index units).
bool taylor_rows(int degree, int dim, Cell centre, const int lo[3], const int hi[3],
                 const std::vector<Vec3>& targets, std::vector<Row>* rows, std::string* err) {
  const auto st = taylor_stencil(degree, dim, centre, lo, hi);
  std::vector<Vec3> offs;
  int ci = -1;
  for (size_t q = 0; q < st.size(); ++q) {
    offs.push_back({(long double)(std::get<0>(st[q]) - std::get<0>(centre)),
                    (long double)(std::get<1>(st[q]) - std::get<1>(centre)),
                    (long double)(std::get<2>(st[q]) - std::get<2>(centre))});
    if (st[q] == centre) ci = (int)q;
  }
  if (ci < 0) {
    *err = "expansion cell outside its stencil";
    return false;
  }
  std::vector<std::vector<long double>> W;
  if (!pinned_fit(offs, ci, degree, dim, targets, &W, err)) return false;
  rows->clear();
  for (size_t t = 0; t < targets.size(); ++t) {
    Row r;
    const bool coincident = targets[t][0] == 0 && targets[t][1] == 0 && targets[t][2] == 0;
    if (coincident) {
      r[centre] = 1.0L;  // the pinned constant
    } else {
      for (size_t q = 0; q < st.size(); ++q) r[st[q]] += W[t][q];
    }
    rows->push_back(r);
  }
  return true;
}

// 1D linear weights at coordinate x (in index units) on centres lo..hi, with
// linear extrapolation from the end pair beyond them; x = num / den exactly.
std::map<int, long double> linear_1d(long num, long den, int lo, int hi) {
  std::map<int, long double> w;
  if (num % den == 0 && num / den >= lo && num / den <= hi) {
    w[(int)(num / den)] = 1.0L;
    return w;
  }
  long fl = num >= 0 ? num / den : -((-num + den - 1) / den);  // floor
  const int a = (int)std::min<long>(std::max<long>(fl, lo), hi - 1);
  const long double t = (long double)(num - (long)a * den) / (long double)den;
  w[a] = 1.0L - t;
  w[a + 1] = t;
  return w;
}

// Rows of one block (direction, scheme) for the anchor column (ab, ac); in two
// dimensions ac = 0 and there is no third axis.
bool block_rows(const ft_operator* op, int ab, int ac, std::vector<Row>* rows, std::string* err) {
  const int p = op->p, k = op->k, dim = op->dim;
  const int lo[3] = {-k, 0, 0};
  const int hi[3] = {k - 1, p - 1, dim == 3 ? p - 1 : 0};
  const int tcn = dim == 3 ? 3 : 1;  // fine columns per coarse column along the third axis
  rows->clear();
  if (op->direction == 0) {
    // Interpolation: expansion cell = containing coarse cell (n = 0, ab, ac);
    // row (g, tb, tc) is the fine ghost centre at offset ((g-1)/3, (tb-1)/3,
    // (tc-1)/3) coarse widths from it (no tc in two dimensions).
    std::vector<Vec3> targets;
    for (int g = 0; g < k; ++g)
      for (int tb = 0; tb < 3; ++tb)
        for (int tc = 0; tc < tcn; ++tc)
          targets.push_back({(long double)(g - 1) / 3.0L, (long double)(tb - 1) / 3.0L,
                             dim == 3 ? (long double)(tc - 1) / 3.0L : 0.0L});
    if (op->scheme == FT_DLINEAR) {
      for (int g = 0; g < k; ++g)
        for (int tb = 0; tb < 3; ++tb)
          for (int tc = 0; tc < tcn; ++tc) {
            const auto wn = linear_1d(g - 1, 3, lo[0], hi[0]);
            const auto wb = linear_1d(3L * ab + tb - 1, 3, 0, p - 1);
            std::map<int, long double> wc;
            if (dim == 3) wc = linear_1d(3L * ac + tc - 1, 3, 0, p - 1); else wc[0] = 1.0L;
            Row r;
            for (auto& [i0, w0] : wn)
              for (auto& [i1, w1] : wb)
                for (auto& [i2, w2] : wc) r[Cell(i0, i1, i2)] += w0 * w1 * w2;
            rows->push_back(r);
          }
      return true;
    }
    return taylor_rows(op->scheme, dim, Cell(0, ab, ac), lo, hi, targets, rows, err);
  }
  // Restriction: coarse target layer l (centre 3l + 3/2 fine widths into the
  // fine side); its nearest fine cell is layer min(3l+1, k-1) of the
  // coincident column (ab, ac) = (3 mu + 1) along b (and c).
  // Averaging along a tangential axis: the three fine columns under the
  // coarse column when all belong to this fine face, else (p not a multiple
  // of 3, the coarse column straddles two fine faces) the one through its
  // centre.
  auto tangential = [&](int j, bool axis_exists) {
    std::map<int, long double> w;
    if (!axis_exists) {
      w[0] = 1.0L;
    } else if (j >= 1 && j + 1 <= p - 1) {
      for (int d = -1; d <= 1; ++d) w[d] = 1.0L / 3.0L;
    } else {
      w[0] = 1.0L;
    }
    return w;
  };
  const auto wtb = tangential(ab, true);
  const auto wtc = tangential(ac, dim == 3);
  for (int l = 0; l < k; ++l) {
    const int eta = std::min(3 * l + 1, k - 1);
    if (op->scheme == FT_DLINEAR) {
      std::map<int, long double> wn;
      if (3 * l + 2 <= k - 1) {
        for (int i = 0; i < 3; ++i) wn[3 * l + i] = 1.0L / 3.0L;
      } else {
        const long double t = (long double)(3 * l + 1 - (k - 2));
        wn[k - 2] = 1.0L - t;
        wn[k - 1] = t;
      }
      Row r;
      for (auto& [i0, w0] : wn)
        for (auto& [db, w1] : wtb)
          for (auto& [dc, w2] : wtc) r[Cell(i0, ab + db, ac + dc)] += w0 * w1 * w2;
      rows->push_back(r);
    } else {
      std::vector<Row> one;
      const std::vector<Vec3> tgt = {{(long double)(3 * l + 1 - eta), 0.0L, 0.0L}};
      if (!taylor_rows(op->scheme, dim, Cell(eta, ab, ac), lo, hi, tgt, &one, err)) return false;
      rows->push_back(one[0]);
    }
  }
  return true;
}

}  // namespace

std::string build_tables(ft_operator* op) {
  const int p = op->p, k = op->k, dim = op->dim;
  op->E = anchors_per_axis(op->direction, p);
  op->R = op->direction == 0 ? (dim == 3 ? 9 : 3) * k : k;
  op->copy_row = -1;
  op->copy_n = 0;
  if (op->direction == 0) {
    // (g, tb, tc) = (1, 1, 1) (3D) or (g, tb) = (1, 1) (2D): the coarse centre
    // itself; with k = 1 no fine ghost centre coincides with a coarse one
    op->copy_row = k >= 2 ? (dim == 3 ? 13 : 4) : -1;
    op->copy_n = 0;
  } else if (op->scheme != FT_DLINEAR) {
    op->copy_row = 0;  // layer 0 coincides with fine layer 1 (k >= 2)
    op->copy_n = 1;
  }
  // Representative anchor column of each axis class.
  int rep[kAxisClasses];
  for (int i = 0; i < kAxisClasses; ++i) rep[i] = -1;
  // Anchor columns that occur: every coarse column (interpolation), or every
  // fine column that coincides with a coarse centre on some subface
  // (restriction; 3m + 1 for multiples of 3, any column otherwise).
  for (int sd = 0; sd < 3; ++sd)
    for (int e = 0; e < op->E; ++e) {
      int m;
      if (op->direction == 0) {
        m = interp_anchor0(sd, p) + e;
        if (!interp_anchor_valid(m, sd, p)) continue;
      } else {
        const int mc = restrict_anchor0(sd, p) + e;
        if (!restrict_anchor_valid(mc, sd, p)) continue;
        m = 3 * mc + 1 - sd * p;
      }
      const int c = axis_class(m, p);
      if (rep[c] < 0) rep[c] = m;
    }
  // Two dimensions: one class per anchor along b, stored at slot cb * 5.
  for (int cb = 0; cb < kAxisClasses; ++cb)
    for (int cc = 0; cc < kAxisClasses; ++cc) {
      HostBlock& blk = op->blocks[cb * kAxisClasses + cc];
      blk = HostBlock();
      if (dim == 2 && cc != 0) continue;
      if (rep[cb] < 0 || (dim == 3 && rep[cc] < 0)) continue;
      const int ab = rep[cb], ac = dim == 3 ? rep[cc] : 0;
      std::vector<Row> rows;
      std::string err;
      if (!block_rows(op, ab, ac, &rows, &err)) return err;
      // Union of source cells with a nonzero weight, ordered (n, c, b), except
      // that the source of the exact-copy row (if any) comes first: the
      // kernels take the copied value from the first loaded stencil point.
      std::map<std::tuple<int, int, int>, int> index;  // key (n, dc, db)
      for (auto& r : rows)
        for (auto& [cell, w] : r)
          if (w != 0.0L)
            index[{std::get<0>(cell), std::get<2>(cell) - ac, std::get<1>(cell) - ab}] = 0;
      int q = 0;
      const std::tuple<int, int, int> copy_key{op->copy_n, 0, 0};
      if (op->copy_row >= 0) {
        if (!index.count(copy_key)) return "internal: copy source missing from its block";
        index[copy_key] = q++;
      }
      for (auto& kv : index)
        if (!(op->copy_row >= 0 && kv.first == copy_key)) kv.second = q++;
      if (q > kMaxStencil) return "weight block wider than supported";
      blk.width = q;
      blk.points.resize(q);
      for (auto& [key, qi] : index)
        blk.points[qi] = pack_point(std::get<0>(key), std::get<2>(key), std::get<1>(key));
      blk.weights.assign((size_t)q * op->R, 0.0);
      for (int r = 0; r < op->R; ++r)
        for (auto& [cell, w] : rows[r]) {
          if (w == 0.0L) continue;
          const int qi = index[{std::get<0>(cell), std::get<2>(cell) - ac, std::get<1>(cell) - ab}];
          blk.weights[(size_t)qi * op->R + r] = (double)w;
        }
      if (op->copy_row >= 0) {
        // The copy row must be exactly one unit weight on (copy_n, anchor).
        const auto& cr = rows[op->copy_row];
        if (cr.size() != 1 || cr.begin()->second != 1.0L ||
            cr.begin()->first != Cell(op->copy_n, ab, ac))
          return "internal: copy row is not an exact copy";
      }
    }
  return "";
}

}  // namespace ft
