// Galerkin assembly of the subdomain stiffness blocks and loads (Eq. discrMS).
//
// Curl-conforming multipatch space (Section 2): on each patch the reference
// basis of component c is D_i(x_c) N_j(x_u) N_k(x_v), with N the degree-p
// B-splines of an open uniform knot vector and D_i = p/(t_{i+p+1}-t_{i+1})
// N_{i+1,p-1} the derived splines; functions are mapped by the covariant
// Piola transform, so curl w = DF curl_hat w_hat / det DF.  Element
// integrals use Gauss-Legendre with p+1 points per direction.
//
// Nonzero B-splines on a knot span are evaluated with the triangular
// Cox-de Boor scheme (Piegl & Tiller, The NURBS Book, Alg. A2.2).
#include <algorithm>
#include <cmath>
#include <string>
#include <vector>

#include "model.hpp"

namespace ieti {

namespace {

struct Basis1D {
  int p, n_el, nq;
  std::vector<double> knots;  // open uniform
  std::vector<double> xq, wq; // per element, nq points mapped to [0,1] (global)
  // tables [e][q][m]
  std::vector<double> N, dN, D;

  void build(int p_, int n_el_) {
    p = p_;
    n_el = n_el_;
    nq = p + 1;
    const int n = n_el + p;
    knots.assign(n + p + 1, 0.0);
    for (int i = 0; i < int(knots.size()); ++i) {
      if (i <= p) knots[i] = 0.0;
      else if (i >= n) knots[i] = 1.0;
      else knots[i] = double(i - p) / n_el;
    }
    // Gauss-Legendre nodes on [-1,1] by Newton on P_nq
    std::vector<double> gx(nq), gw(nq);
    for (int i = 0; i < nq; ++i) {
      double x = std::cos(M_PI * (i + 0.75) / (nq + 0.5));
      for (int it = 0; it < 100; ++it) {
        double p0 = 1.0, p1 = x;
        for (int k = 2; k <= nq; ++k) {
          double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
          p0 = p1;
          p1 = p2;
        }
        double pn = (nq == 1) ? x : p1;
        double pm = (nq == 1) ? 1.0 : p0;
        double dp = nq * (x * pn - pm) / (x * x - 1.0);
        double dx = pn / dp;
        x -= dx;
        if (std::fabs(dx) < 1e-16) break;
      }
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= nq; ++k) {
        double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      double pn = (nq == 1) ? x : p1;
      double pm = (nq == 1) ? 1.0 : p0;
      double dp = nq * (x * pn - pm) / (x * x - 1.0);
      gx[i] = x;
      gw[i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    xq.resize(n_el * nq);
    wq.resize(n_el * nq);
    N.assign(n_el * nq * (p + 1), 0.0);
    dN.assign(n_el * nq * (p + 1), 0.0);
    D.assign(n_el * nq * p, 0.0);
    std::vector<double> lo(p + 1), hi(p + 1), left(p + 2), right(p + 2);
    for (int e = 0; e < n_el; ++e) {
      const int s = p + e;  // knot span
      const double a = knots[s], b = knots[s + 1];
      for (int q = 0; q < nq; ++q) {
        const double x = a + 0.5 * (gx[q] + 1.0) * (b - a);
        xq[e * nq + q] = x;
        wq[e * nq + q] = 0.5 * gw[q] * (b - a);
        // degree p-1 and p nonzero functions on span s
        auto eval = [&](int deg, std::vector<double>& out) {
          out.assign(deg + 1, 0.0);
          out[0] = 1.0;
          for (int j = 1; j <= deg; ++j) {
            left[j] = x - knots[s + 1 - j];
            right[j] = knots[s + j] - x;
            double saved = 0.0;
            for (int r = 0; r < j; ++r) {
              double tmp = out[r] / (right[r + 1] + left[j - r]);
              out[r] = saved + right[r + 1] * tmp;
              saved = left[j - r] * tmp;
            }
            out[j] = saved;
          }
        };
        eval(p - 1, lo);  // N_{s-p+1+m, p-1}, m = 0..p-1
        eval(p, hi);      // N_{s-p+m, p},     m = 0..p
        double* Nrow = &N[(e * nq + q) * (p + 1)];
        double* dNrow = &dN[(e * nq + q) * (p + 1)];
        double* Drow = &D[(e * nq + q) * p];
        for (int m = 0; m <= p; ++m) Nrow[m] = hi[m];
        // D_i for i = s-p+m (m = 0..p-1) uses N_{i+1,p-1} = lo[m]
        for (int m = 0; m < p; ++m) {
          const int i = s - p + m;
          Drow[m] = p / (knots[i + p + 1] - knots[i + 1]) * lo[m];
        }
        // N'_i = D_{i-1} - D_i
        for (int m = 0; m <= p; ++m) {
          double v = 0.0;
          if (m >= 1) v += Drow[m - 1];
          if (m < p) v -= Drow[m];
          dNrow[m] = v;
        }
      }
    }
  }
};

// Geometry map of one patch: point and Jacobian DF[a][b] = dx_a/dxi_b.
void patch_map(const ieti_problem& pr, int64_t q, const double xi[3], double x[3], double DF[3][3]) {
  const int P0 = pr.patches[0], P1 = pr.patches[1], P2 = pr.patches[2];
  const int64_t i = q % P0, j = (q / P0) % P1, k = q / (int64_t(P0) * P1);
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) DF[a][b] = 0.0;
  const double* g = pr.geom_params;
  if (pr.geom_kind == IETI_GEOM_BOX) {
    const double h[3] = {(g[1] - g[0]) / P0, (g[3] - g[2]) / P1, (g[5] - g[4]) / P2};
    const int64_t c[3] = {i, j, k};
    const double lo[3] = {g[0], g[2], g[4]};
    for (int a = 0; a < 3; ++a) {
      x[a] = lo[a] + h[a] * (double(c[a]) + xi[a]);
      DF[a][a] = h[a];
    }
    return;
  }
  // annulus: rational quadratic arc per sector
  const double dth = 2.0 * M_PI / P0;
  const double t0 = i * dth, half = 0.5 * dth, w1 = std::cos(half);
  const double cx[3] = {std::cos(t0), std::cos(t0 + half) / w1, std::cos(t0 + dth)};
  const double cy[3] = {std::sin(t0), std::sin(t0 + half) / w1, std::sin(t0 + dth)};
  const double w[3] = {1.0, w1, 1.0};
  const double s = xi[0];
  const double B[3] = {(1 - s) * (1 - s), 2 * s * (1 - s), s * s};
  const double dB[3] = {-2 * (1 - s), 2 - 4 * s, 2 * s};
  double W = 0, dW = 0, nx = 0, ny = 0, dnx = 0, dny = 0;
  for (int m = 0; m < 3; ++m) {
    W += w[m] * B[m];
    dW += w[m] * dB[m];
    nx += w[m] * cx[m] * B[m];
    ny += w[m] * cy[m] * B[m];
    dnx += w[m] * cx[m] * dB[m];
    dny += w[m] * cy[m] * dB[m];
  }
  const double ux = nx / W, uy = ny / W;
  const double dux = (dnx * W - nx * dW) / (W * W), duy = (dny * W - ny * dW) / (W * W);
  const double r0 = g[2 + j], r1 = g[3 + j];
  const double r = r0 + xi[1] * (r1 - r0);
  const double hz = (g[1] - g[0]) / P2;
  x[0] = r * ux;
  x[1] = r * uy;
  x[2] = g[0] + (double(k) + xi[2]) * hz;
  DF[0][0] = r * dux;
  DF[1][0] = r * duy;
  DF[0][1] = (r1 - r0) * ux;
  DF[1][1] = (r1 - r0) * uy;
  DF[2][2] = hz;
}

// Boundary L2 projection of n x A_D: boundary DOFs a_D with
// sum_e a_e int (w_e)_t . (w_f)_t dS = int (A_D)_t . (w_f)_t dS for every
// boundary function f, over the patch faces on the boundary of the domain.
// Only the two tangential components with index 0 (or last) across the face
// have a tangential trace there (open knots; the normal component's
// push-forward DF^{-T} e_d is normal to the face).  The mass system is
// solved by Jacobi-preconditioned CG.  aD is indexed by global edge id.
int dirichlet_projection(const Model& m, const Basis1D& bs, std::vector<double>& aD, Error& err) {
  const Mesh& M = m.mesh;
  const int p = M.p, n = M.n, n1 = n - 1, ne = M.n_el, nq = bs.nq;
  const int64_t n_patches = int64_t(M.P[0]) * M.P[1] * M.P[2];
  struct Face {
    int64_t q;
    int d, side;
  };
  std::vector<Face> faces;
  for (int64_t q = 0; q < n_patches; ++q) {
    const int64_t pc[3] = {q % M.P[0], (q / M.P[0]) % M.P[1], q / (int64_t(M.P[0]) * M.P[1])};
    for (int d = 0; d < 3; ++d) {
      if (M.per[d]) continue;
      if (pc[d] == 0) faces.push_back({q, d, 0});
      if (pc[d] == M.P[d] - 1) faces.push_back({q, d, 1});
    }
  }
  const int64_t per_face = int64_t(ne) * ne * nq * nq;
  // points of every face (element-major, then Gauss points; axis a fastest)
  std::vector<double> pts(size_t(faces.size()) * per_face * 3), dfs(size_t(faces.size()) * per_face * 9);
  for (size_t f = 0; f < faces.size(); ++f) {
    const int d = faces[f].d, a = (d + 1) % 3 < (d + 2) % 3 ? (d + 1) % 3 : (d + 2) % 3;
    const int b = 3 - d - a;
    for (int64_t t = 0; t < per_face; ++t) {
      const int qa = int(t % nq), qb = int((t / nq) % nq), ea = int((t / (nq * nq)) % ne), eb = int(t / (int64_t(nq) * nq * ne));
      double xi[3], x[3], DF[3][3];
      xi[a] = bs.xq[ea * nq + qa];
      xi[b] = bs.xq[eb * nq + qb];
      xi[d] = double(faces[f].side);
      patch_map(m.prob, faces[f].q, xi, x, DF);
      for (int c = 0; c < 3; ++c) pts[(f * per_face + t) * 3 + c] = x[c];
      for (int r = 0; r < 9; ++r) dfs[(f * per_face + t) * 9 + r] = DF[r / 3][r % 3];
    }
  }
  std::vector<double> Ad(pts.size(), 0.0);
  m.prob.A_D(pts.data(), int64_t(pts.size() / 3), Ad.data(), m.prob.A_D_user);
  for (double v : Ad)
    if (!std::isfinite(v)) {
      err = {IETI_ERR_INVALID_ARG, "Dirichlet data returned a non-finite value"};
      return err.code;
    }
  // element face matrices -> global triplets over Dirichlet edges
  std::vector<int64_t> pos(M.n_edges, -1), dofs;
  for (int64_t e = 0; e < M.n_edges; ++e)
    if (m.dirichlet[e]) {
      pos[e] = int64_t(dofs.size());
      dofs.push_back(e);
    }
  const int64_t nD = int64_t(dofs.size());
  struct T3 {
    int64_t r, c;
    double v;
  };
  std::vector<T3> trip;
  std::vector<double> rhs(nD, 0.0);
  const int nfe = 2 * p * (p + 1);
  std::vector<int64_t> fid(nfe);
  std::vector<double> wt(size_t(nfe) * 3), Me(size_t(nfe) * nfe), be(nfe);
  for (size_t f = 0; f < faces.size(); ++f) {
    const int d = faces[f].d, a = (d + 1) % 3 < (d + 2) % 3 ? (d + 1) % 3 : (d + 2) % 3;
    const int b = 3 - d - a;
    const int64_t q = faces[f].q;
    const int64_t pc[3] = {q % M.P[0], (q / M.P[0]) % M.P[1], q / (int64_t(M.P[0]) * M.P[1])};
    for (int ea = 0; ea < ne; ++ea)
      for (int eb = 0; eb < ne; ++eb) {
        // element face functions: component c in {a, b}, active indices along a and b
        int k = 0;
        for (int c : {a, b}) {
          const int ma = (a == c) ? p : p + 1, mb = (b == c) ? p : p + 1;
          for (int ib = 0; ib < mb; ++ib)
            for (int ia = 0; ia < ma; ++ia, ++k) {
              int64_t idx[3];
              idx[a] = ea + ia;
              idx[b] = eb + ib;
              idx[d] = faces[f].side == 0 ? 0 : n - 1;  // c != d: n functions across the face
              fid[k] = pos[M.edge_id(c, M.wrap(0, pc[0] * n1 + idx[0]), M.wrap(1, pc[1] * n1 + idx[1]),
                                     M.wrap(2, pc[2] * n1 + idx[2]))];
              if (fid[k] < 0) {
                err = {IETI_ERR_TREE, "a boundary face function is not a Dirichlet DOF"};
                return err.code;
              }
            }
        }
        std::fill(Me.begin(), Me.end(), 0.0);
        std::fill(be.begin(), be.end(), 0.0);
        for (int qb = 0; qb < nq; ++qb)
          for (int qa = 0; qa < nq; ++qa) {
            const int64_t t = qa + nq * (qb + int64_t(nq) * (ea + int64_t(ne) * eb));
            const double* D9 = &dfs[(f * per_face + t) * 9];
            double DF[3][3];
            for (int r = 0; r < 9; ++r) DF[r / 3][r % 3] = D9[r];
            const double det = DF[0][0] * (DF[1][1] * DF[2][2] - DF[1][2] * DF[2][1]) -
                               DF[0][1] * (DF[1][0] * DF[2][2] - DF[1][2] * DF[2][0]) +
                               DF[0][2] * (DF[1][0] * DF[2][1] - DF[1][1] * DF[2][0]);
            // columns of DF^{-T}: G[:, c] = cof(DF)[:, c] / det
            double G[3][3];
            G[0][0] = (DF[1][1] * DF[2][2] - DF[1][2] * DF[2][1]) / det;
            G[0][1] = -(DF[1][0] * DF[2][2] - DF[1][2] * DF[2][0]) / det;
            G[0][2] = (DF[1][0] * DF[2][1] - DF[1][1] * DF[2][0]) / det;
            G[1][0] = -(DF[0][1] * DF[2][2] - DF[0][2] * DF[2][1]) / det;
            G[1][1] = (DF[0][0] * DF[2][2] - DF[0][2] * DF[2][0]) / det;
            G[1][2] = -(DF[0][0] * DF[2][1] - DF[0][1] * DF[2][0]) / det;
            G[2][0] = (DF[0][1] * DF[1][2] - DF[0][2] * DF[1][1]) / det;
            G[2][1] = -(DF[0][0] * DF[1][2] - DF[0][2] * DF[1][0]) / det;
            G[2][2] = (DF[0][0] * DF[1][1] - DF[0][1] * DF[1][0]) / det;
            const double nv[3] = {G[0][d], G[1][d], G[2][d]};
            const double nl = std::sqrt(nv[0] * nv[0] + nv[1] * nv[1] + nv[2] * nv[2]);
            const double nh[3] = {nv[0] / nl, nv[1] / nl, nv[2] / nl};
            const double dS = bs.wq[ea * nq + qa] * bs.wq[eb * nq + qb] * std::fabs(det) * nl;
            int kk = 0;
            for (int c : {a, b}) {
              const int ma = (a == c) ? p : p + 1, mb = (b == c) ? p : p + 1;
              for (int ib = 0; ib < mb; ++ib)
                for (int ia = 0; ia < ma; ++ia, ++kk) {
                  const double fa = (a == c) ? bs.D[(ea * nq + qa) * p + ia] : bs.N[(ea * nq + qa) * (p + 1) + ia];
                  const double fb = (b == c) ? bs.D[(eb * nq + qb) * p + ib] : bs.N[(eb * nq + qb) * (p + 1) + ib];
                  const double sv = fa * fb;
                  double w[3] = {G[0][c] * sv, G[1][c] * sv, G[2][c] * sv};
                  const double wn = w[0] * nh[0] + w[1] * nh[1] + w[2] * nh[2];
                  for (int r = 0; r < 3; ++r) wt[kk * 3 + r] = w[r] - wn * nh[r];
                }
            }
            const double* A = &Ad[(f * per_face + t) * 3];
            for (int i = 0; i < nfe; ++i) {
              const double* wi = &wt[i * 3];
              be[i] += dS * (A[0] * wi[0] + A[1] * wi[1] + A[2] * wi[2]);
              for (int j = 0; j < nfe; ++j) {
                const double* wj = &wt[j * 3];
                Me[size_t(i) * nfe + j] += dS * (wi[0] * wj[0] + wi[1] * wj[1] + wi[2] * wj[2]);
              }
            }
          }
        for (int i = 0; i < nfe; ++i) {
          rhs[fid[i]] += be[i];
          for (int j = 0; j < nfe; ++j)
            if (Me[size_t(i) * nfe + j] != 0.0) trip.push_back({fid[i], fid[j], Me[size_t(i) * nfe + j]});
        }
      }
  }
  // CSR (duplicates summed in a fixed order)
  std::sort(trip.begin(), trip.end(), [](const T3& x, const T3& y) { return x.r != y.r ? x.r < y.r : x.c < y.c; });
  std::vector<int64_t> ptr(nD + 1, 0), col;
  std::vector<double> val;
  for (size_t i = 0; i < trip.size();) {
    size_t j = i;
    double v = 0.0;
    while (j < trip.size() && trip[j].r == trip[i].r && trip[j].c == trip[i].c) v += trip[j++].v;
    col.push_back(trip[i].c);
    val.push_back(v);
    ptr[trip[i].r + 1]++;
    i = j;
  }
  for (int64_t r = 0; r < nD; ++r) ptr[r + 1] += ptr[r];
  std::vector<double> dg(nD, 0.0);
  for (int64_t r = 0; r < nD; ++r)
    for (int64_t k = ptr[r]; k < ptr[r + 1]; ++k)
      if (col[k] == r) dg[r] = val[k];
  for (int64_t r = 0; r < nD; ++r)
    if (!(dg[r] > 0.0)) {
      err = {IETI_ERR_TREE, "a Dirichlet DOF has no tangential trace on the boundary"};
      return err.code;
    }
  auto matvec = [&](const std::vector<double>& x, std::vector<double>& y) {
    for (int64_t r = 0; r < nD; ++r) {
      double s = 0.0;
      for (int64_t k = ptr[r]; k < ptr[r + 1]; ++k) s += val[k] * x[col[k]];
      y[r] = s;
    }
  };
  std::vector<double> x(nD, 0.0), r = rhs, z(nD), pv(nD), Ap(nD);
  double bnorm = 0.0;
  for (double v : rhs) bnorm += v * v;
  bnorm = std::sqrt(bnorm);
  for (int64_t i = 0; i < nD; ++i) z[i] = r[i] / dg[i];
  pv = z;
  double rz = 0.0;
  for (int64_t i = 0; i < nD; ++i) rz += r[i] * z[i];
  const int max_it = int(std::min<int64_t>(20 * nD + 100, 1000000));
  bool conv = bnorm == 0.0;
  for (int it = 0; it < max_it && !conv; ++it) {
    matvec(pv, Ap);
    double pAp = 0.0;
    for (int64_t i = 0; i < nD; ++i) pAp += pv[i] * Ap[i];
    const double al = rz / pAp;
    double rr = 0.0;
    for (int64_t i = 0; i < nD; ++i) {
      x[i] += al * pv[i];
      r[i] -= al * Ap[i];
      rr += r[i] * r[i];
    }
    if (std::sqrt(rr) <= 1e-15 * bnorm) {
      conv = true;
      break;
    }
    double rz2 = 0.0;
    for (int64_t i = 0; i < nD; ++i) {
      z[i] = r[i] / dg[i];
      rz2 += r[i] * z[i];
    }
    const double be2 = rz2 / rz;
    rz = rz2;
    for (int64_t i = 0; i < nD; ++i) pv[i] = z[i] + be2 * pv[i];
  }
  if (!conv) {
    err = {IETI_ERR_NOT_CONVERGED, "the boundary projection of the Dirichlet data did not converge"};
    return err.code;
  }
  aD.assign(M.n_edges, 0.0);
  for (int64_t i = 0; i < nD; ++i) aD[dofs[i]] = x[i];
  return IETI_OK;
}

}  // namespace

int assemble_local_systems(Model& m, Error& err) {
  const Mesh& M = m.mesh;
  const int p = M.p, n = M.n, n1 = n - 1, ne1 = M.n_el;
  Basis1D bs;
  bs.build(p, M.n_el);
  const int nq = bs.nq;
  const int Q = nq * nq * nq;
  const int nfc[3] = {p * (p + 1) * (p + 1), p * (p + 1) * (p + 1), p * (p + 1) * (p + 1)};
  const int nf = nfc[0] + nfc[1] + nfc[2];
  const int64_t n_patches = int64_t(M.P[0]) * M.P[1] * M.P[2];
  const int64_t n_elem = int64_t(ne1) * ne1 * ne1;
  // patch-local numbering: component c, indices (i0,i1,i2), i0 fastest;
  // local extents le[c][a] = n-1 along a == c, else n.
  int64_t base[4] = {0, 0, 0, 0};
  for (int c = 0; c < 3; ++c) base[c + 1] = base[c] + int64_t(n1) * n * n;
  const int64_t nloc = base[3];

  // global edge id -> subdomain-local index over [r, p] (per subdomain)
  // stored per patch: local patch function -> (subdomain-local index or -1)
  // ---- quadrature points of every patch, and J there (caller callback)
  std::vector<double> Jval;
  {
    std::vector<double> pts(size_t(n_patches) * n_elem * Q * 3);
    for (int64_t q = 0; q < n_patches; ++q)
      for (int64_t el = 0; el < n_elem; ++el) {
        const int e0 = int(el % ne1), e1 = int((el / ne1) % ne1), e2 = int(el / (int64_t(ne1) * ne1));
        for (int t = 0; t < Q; ++t) {
          const int q0 = t % nq, q1 = (t / nq) % nq, q2 = t / (nq * nq);
          double xi[3] = {bs.xq[e0 * nq + q0], bs.xq[e1 * nq + q1], bs.xq[e2 * nq + q2]};
          double x[3], DF[3][3];
          patch_map(m.prob, q, xi, x, DF);
          double* o = &pts[((q * n_elem + el) * Q + t) * 3];
          o[0] = x[0];
          o[1] = x[1];
          o[2] = x[2];
        }
      }
    Jval.assign(pts.size(), 0.0);
    const int64_t npts = int64_t(pts.size() / 3);
    m.prob.J(pts.data(), npts, Jval.data(), m.prob.J_user);
  }

  // ---- local index of every edge in each subdomain's [r, p] numbering
  std::vector<std::vector<int32_t>> sub_index(m.n_sub);
  // use a sorted lookup per subdomain (r then p)
  auto local_of = [&](int k, int64_t e) -> int32_t {
    const Subdomain& s = m.sd[k];
    auto it = std::lower_bound(s.r_edges.begin(), s.r_edges.end(), e);
    if (it != s.r_edges.end() && *it == e) return int32_t(it - s.r_edges.begin());
    auto jt = std::lower_bound(s.p_edges.begin(), s.p_edges.end(), e);
    if (jt != s.p_edges.end() && *jt == e) return int32_t(s.r_edges.size() + (jt - s.p_edges.begin()));
    return -1;
  };

  // triplets per subdomain
  struct Trip {
    int32_t r, c;
    int32_t patch;
    double v;
  };
  std::vector<std::vector<Trip>> trips(m.n_sub);
  for (int k = 0; k < m.n_sub; ++k) {
    m.sd[k].n_loc = int64_t(m.sd[k].r_edges.size() + m.sd[k].p_edges.size());
    m.sd[k].load.assign(m.sd[k].n_loc, 0.0);
  }

  // non-homogeneous Dirichlet data: prescribed boundary coefficients
  std::vector<double> aD;
  const bool lift = m.prob.A_D != nullptr;
  m.d_edges.clear();
  m.d_vals.clear();
  if (lift) {
    if (int rc = dirichlet_projection(m, bs, aD, err)) return rc;
    for (int64_t e = 0; e < M.n_edges; ++e)
      if (m.dirichlet[e]) {
        m.d_edges.push_back(e);
        m.d_vals.push_back(aD[e]);
      }
  }

  int failed = 0;
  std::vector<std::vector<std::pair<int32_t, double>>> patch_load(n_patches), patch_lift(n_patches);
#pragma omp parallel
  {
    std::vector<double> Kp;       // dense patch matrix (nu = 1)
    std::vector<double> jp;       // patch load
    std::vector<int32_t> fidx(nf);  // patch-local index of element functions
    std::vector<double> curl(size_t(Q) * nf * 3), val(size_t(Q) * nf * 3), W(Q);
    std::vector<double> Ke(size_t(nf) * nf), je(nf);
    std::vector<int64_t> gid(nloc);
    std::vector<int32_t> lid(nloc);
    std::vector<Trip> local_trips;
#pragma omp for schedule(dynamic, 1)
    for (int64_t q = 0; q < n_patches; ++q) {
      const int k = m.part[q];
      const int64_t pc[3] = {q % M.P[0], (q / M.P[0]) % M.P[1], q / (int64_t(M.P[0]) * M.P[1])};
      // local -> global edge ids and subdomain-local ids
      for (int c = 0; c < 3; ++c) {
        const int64_t le[3] = {c == 0 ? n1 : n, c == 1 ? n1 : n, c == 2 ? n1 : n};
        for (int64_t i2 = 0; i2 < le[2]; ++i2)
          for (int64_t i1 = 0; i1 < le[1]; ++i1)
            for (int64_t i0 = 0; i0 < le[0]; ++i0) {
              const int64_t li = base[c] + i0 + le[0] * (i1 + le[1] * i2);
              const int64_t e = M.edge_id(c, M.wrap(0, pc[0] * n1 + i0), M.wrap(1, pc[1] * n1 + i1),
                                          M.wrap(2, pc[2] * n1 + i2));
              gid[li] = e;
              lid[li] = (m.dirichlet[e] || m.tree[e]) ? -1 : local_of(k, e);
            }
      }
      Kp.assign(size_t(nloc) * nloc, 0.0);
      jp.assign(nloc, 0.0);
      for (int64_t el = 0; el < n_elem; ++el) {
        const int e[3] = {int(el % ne1), int((el / ne1) % ne1), int(el / (int64_t(ne1) * ne1))};
        // element function indices
        int f = 0;
        for (int c = 0; c < 3; ++c) {
          const int m0 = (c == 0) ? p : p + 1, m1 = (c == 1) ? p : p + 1, m2 = (c == 2) ? p : p + 1;
          const int64_t le[3] = {c == 0 ? n1 : n, c == 1 ? n1 : n, c == 2 ? n1 : n};
          for (int a2 = 0; a2 < m2; ++a2)
            for (int a1 = 0; a1 < m1; ++a1)
              for (int a0 = 0; a0 < m0; ++a0)
                fidx[f++] = int32_t(base[c] + (e[0] + a0) + le[0] * ((e[1] + a1) + le[1] * (e[2] + a2)));
        }
        for (int t = 0; t < Q; ++t) {
          const int qq[3] = {t % nq, (t / nq) % nq, t / (nq * nq)};
          double xi[3], x[3], DF[3][3];
          for (int a = 0; a < 3; ++a) xi[a] = bs.xq[e[a] * nq + qq[a]];
          patch_map(m.prob, q, xi, x, DF);
          const double det = DF[0][0] * (DF[1][1] * DF[2][2] - DF[1][2] * DF[2][1]) -
                             DF[0][1] * (DF[1][0] * DF[2][2] - DF[1][2] * DF[2][0]) +
                             DF[0][2] * (DF[1][0] * DF[2][1] - DF[1][1] * DF[2][0]);
          // inverse transpose: DF^{-T} = cof(DF)/det
          double cof[3][3];
          cof[0][0] = DF[1][1] * DF[2][2] - DF[1][2] * DF[2][1];
          cof[0][1] = -(DF[1][0] * DF[2][2] - DF[1][2] * DF[2][0]);
          cof[0][2] = DF[1][0] * DF[2][1] - DF[1][1] * DF[2][0];
          cof[1][0] = -(DF[0][1] * DF[2][2] - DF[0][2] * DF[2][1]);
          cof[1][1] = DF[0][0] * DF[2][2] - DF[0][2] * DF[2][0];
          cof[1][2] = -(DF[0][0] * DF[2][1] - DF[0][1] * DF[2][0]);
          cof[2][0] = DF[0][1] * DF[1][2] - DF[0][2] * DF[1][1];
          cof[2][1] = -(DF[0][0] * DF[1][2] - DF[0][2] * DF[1][0]);
          cof[2][2] = DF[0][0] * DF[1][1] - DF[0][1] * DF[1][0];
          double w = bs.wq[e[0] * nq + qq[0]] * bs.wq[e[1] * nq + qq[1]] * bs.wq[e[2] * nq + qq[2]];
          W[t] = w * std::fabs(det);
          const double* Nt[3];
          const double* dNt[3];
          const double* Dt[3];
          for (int a = 0; a < 3; ++a) {
            Nt[a] = &bs.N[(e[a] * nq + qq[a]) * (p + 1)];
            dNt[a] = &bs.dN[(e[a] * nq + qq[a]) * (p + 1)];
            Dt[a] = &bs.D[(e[a] * nq + qq[a]) * p];
          }
          int ff = 0;
          for (int c = 0; c < 3; ++c) {
            const int m0 = (c == 0) ? p : p + 1, m1 = (c == 1) ? p : p + 1, m2 = (c == 2) ? p : p + 1;
            for (int a2 = 0; a2 < m2; ++a2)
              for (int a1 = 0; a1 < m1; ++a1)
                for (int a0 = 0; a0 < m0; ++a0, ++ff) {
                  // values f_a and derivatives g_a of the three 1D factors
                  const double f0 = (c == 0) ? Dt[0][a0] : Nt[0][a0];
                  const double f1 = (c == 1) ? Dt[1][a1] : Nt[1][a1];
                  const double f2 = (c == 2) ? Dt[2][a2] : Nt[2][a2];
                  const double g0 = (c == 0) ? 0.0 : dNt[0][a0];
                  const double g1 = (c == 1) ? 0.0 : dNt[1][a1];
                  const double g2 = (c == 2) ? 0.0 : dNt[2][a2];
                  // reference value s*e_c; reference gradient of s
                  const double s = f0 * f1 * f2;
                  const double ds[3] = {g0 * f1 * f2, f0 * g1 * f2, f0 * f1 * g2};
                  // curl_hat(s e_c) = grad s x e_c
                  double ch[3];
                  if (c == 0) { ch[0] = 0.0; ch[1] = ds[2]; ch[2] = -ds[1]; }
                  else if (c == 1) { ch[0] = -ds[2]; ch[1] = 0.0; ch[2] = ds[0]; }
                  else { ch[0] = ds[1]; ch[1] = -ds[0]; ch[2] = 0.0; }
                  double* cu = &curl[(size_t(t) * nf + ff) * 3];
                  double* va = &val[(size_t(t) * nf + ff) * 3];
                  for (int a = 0; a < 3; ++a) {
                    cu[a] = (DF[a][0] * ch[0] + DF[a][1] * ch[1] + DF[a][2] * ch[2]) / det;
                    va[a] = cof[a][c] * s / det;
                  }
                }
          }
        }
        // element matrix and load
        for (int a = 0; a < nf; ++a) {
          for (int b = a; b < nf; ++b) {
            double acc = 0.0;
            for (int t = 0; t < Q; ++t) {
              const double* ca = &curl[(size_t(t) * nf + a) * 3];
              const double* cb = &curl[(size_t(t) * nf + b) * 3];
              acc += W[t] * (ca[0] * cb[0] + ca[1] * cb[1] + ca[2] * cb[2]);
            }
            Ke[size_t(a) * nf + b] = acc;
            Ke[size_t(b) * nf + a] = acc;
          }
          double acc = 0.0;
          for (int t = 0; t < Q; ++t) {
            const double* va = &val[(size_t(t) * nf + a) * 3];
            const double* J = &Jval[((q * n_elem + el) * Q + t) * 3];
            acc += W[t] * (J[0] * va[0] + J[1] * va[1] + J[2] * va[2]);
          }
          je[a] = acc;
        }
        for (int a = 0; a < nf; ++a) {
          double* row = &Kp[size_t(fidx[a]) * nloc];
          for (int b = 0; b < nf; ++b) row[fidx[b]] += Ke[size_t(a) * nf + b];
          jp[fidx[a]] += je[a];
        }
      }
      // scatter to subdomain triplets (nu applied)
      local_trips.clear();
      for (int64_t a = 0; a < nloc; ++a) {
        if (lid[a] < 0) continue;
        const double* row = &Kp[size_t(a) * nloc];
        for (int64_t b = 0; b < nloc; ++b) {
          if (lid[b] < 0 || row[b] == 0.0) continue;
          local_trips.push_back({lid[a], lid[b], int32_t(q), row[b]});
        }
      }
      auto& PL = patch_load[q];
      for (int64_t a = 0; a < nloc; ++a)
        if (lid[a] >= 0) PL.emplace_back(lid[a], jp[a]);
      if (lift) {
        auto& LF = patch_lift[q];
        for (int64_t a = 0; a < nloc; ++a) {
          if (lid[a] < 0) continue;
          const double* row = &Kp[size_t(a) * nloc];
          double v = 0.0;
          for (int64_t b = 0; b < nloc; ++b)
            if (row[b] != 0.0 && m.dirichlet[gid[b]]) v += row[b] * aD[gid[b]];
          if (v != 0.0) LF.emplace_back(lid[a], v);
        }
      }
#pragma omp critical
      {
        auto& T = trips[k];
        T.insert(T.end(), local_trips.begin(), local_trips.end());
      }
    }
  }
  if (failed) {
    err = {IETI_ERR_INVALID_ARG, "assembly failed"};
    return err.code;
  }
  m.patch_load = std::move(patch_load);
  m.patch_lift = std::move(patch_lift);
  // ---- merge triplets into CSR per subdomain (deterministic order)
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k < m.n_sub; ++k) {
    auto& T = trips[k];
    std::stable_sort(T.begin(), T.end(), [](const Trip& x, const Trip& y) {
      if (x.r != y.r) return x.r < y.r;
      if (x.c != y.c) return x.c < y.c;
      return x.patch < y.patch;
    });
    Subdomain& s = m.sd[k];
    s.indptr.assign(s.n_loc + 1, 0);
    s.indices.clear();
    s.tr_seg.assign(1, 0);
    s.tr_patch.resize(T.size());
    s.tr_val.resize(T.size());
    size_t i = 0;
    while (i < T.size()) {
      size_t j = i;
      while (j < T.size() && T[j].r == T[i].r && T[j].c == T[i].c) {
        s.tr_patch[j] = T[j].patch;
        s.tr_val[j] = T[j].v;
        ++j;
      }
      s.indices.push_back(T[i].c);
      s.tr_seg.push_back(int64_t(j));
      s.indptr[T[i].r + 1]++;
      i = j;
    }
    for (int64_t r = 0; r < s.n_loc; ++r) s.indptr[r + 1] += s.indptr[r];
    std::vector<Trip>().swap(T);
  }
  std::vector<double> ones(n_patches, 1.0);
  return set_coefficients(m, m.nu.data(), ones.data(), err);
}

int set_coefficients(Model& m, const double* nu, const double* load_scale, Error& err) {
  const int64_t n_patches = int64_t(m.part.size());
  for (int64_t q = 0; q < n_patches; ++q)
    if (!(nu[q] > 0.0) || !std::isfinite(nu[q]) || !std::isfinite(load_scale[q])) {
      err = {IETI_ERR_INVALID_ARG, "reluctivity must be positive and finite, load scales finite (patch " +
                                       std::to_string(q) + ")"};
      return err.code;
    }
  if (m.nu.data() != nu) m.nu.assign(nu, nu + n_patches);
  m.load_scale.assign(load_scale, load_scale + n_patches);
#pragma omp parallel for schedule(dynamic, 1)
  for (int k = 0; k < m.n_sub; ++k) {
    Subdomain& s = m.sd[k];
    const int64_t nnz = int64_t(s.tr_seg.size()) - 1;
    s.values.resize(nnz);
    for (int64_t i = 0; i < nnz; ++i) {
      double v = 0.0;
      for (int64_t t = s.tr_seg[i]; t < s.tr_seg[i + 1]; ++t) v += m.nu[s.tr_patch[t]] * s.tr_val[t];
      s.values[i] = v;
    }
    std::fill(s.load.begin(), s.load.end(), 0.0);
  }
  // loads summed in patch order (deterministic)
  for (int64_t q = 0; q < n_patches; ++q) {
    Subdomain& s = m.sd[m.part[q]];
    const double c = m.load_scale[q];
    for (const auto& pr : m.patch_load[q]) s.load[pr.first] += c * pr.second;
    if (!m.patch_lift.empty())
      for (const auto& pr : m.patch_lift[q]) s.load[pr.first] -= m.nu[q] * pr.second;
  }
  return IETI_OK;
}

}  // namespace ieti
