// Host planner: lowering of the brickwork tensor network into the boundary
// tensor schedule (see plan.hpp for the formulation).
#include "plan.hpp"

#include "lds_layout.hpp"

#include <algorithm>
#include <cmath>
#include <cstring>
#include <set>
#include <sstream>

namespace tnc {

namespace {
constexpr int kErrInvalid = -1;
constexpr int kErrDomain = -2;
constexpr int kErrRank = -3;
// The host folds the 2^k x 2^k early-region tensor into the first late
// launch at O(2^(3k)) cost, which bounds k.
constexpr int kMaxOpenLegs = 10;

int fail(std::string* err, int code, const std::string& msg) {
  if (err) *err = msg;
  return code;
}

M2 diag(cd a, cd b) {
  M2 m;
  m.a[0] = a; m.a[1] = 0; m.a[2] = 0; m.a[3] = b;
  return m;
}

M2 inverse(const M2& m) {
  cd det = m.a[0] * m.a[3] - m.a[1] * m.a[2];
  M2 r;
  r.a[0] = m.a[3] / det; r.a[1] = -m.a[1] / det;
  r.a[2] = -m.a[2] / det; r.a[3] = m.a[0] / det;
  return r;
}

cd det2(const M2& m) { return m.a[0] * m.a[3] - m.a[1] * m.a[2]; }

M2 add(const M2& x, const M2& y, cd s = 1.0) {
  M2 r;
  for (int i = 0; i < 4; ++i) r.a[i] = x.a[i] + s * y.a[i];
  return r;
}

// row vector f times matrix m: (f m)[j] = sum_i f[i] m[i][j]
void rowvec_mul(const cd f[2], const M2& m, cd out[2]) {
  out[0] = f[0] * m(0, 0) + f[1] * m(1, 0);
  out[1] = f[0] * m(0, 1) + f[1] * m(1, 1);
}

void mat_vec(const M2& m, const cd v[2], cd out[2]) {
  out[0] = m(0, 0) * v[0] + m(0, 1) * v[1];
  out[1] = m(1, 0) * v[0] + m(1, 1) * v[1];
}

double maxabs(const cd* a, int n) {
  double m = 0;
  for (int i = 0; i < n; ++i) m = std::max(m, std::abs(a[i]));
  return m;
}
}  // namespace

M2 operator*(const M2& x, const M2& y) {
  M2 r;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) r(i, j) = x(i, 0) * y(0, j) + x(i, 1) * y(1, j);
  return r;
}

// ---------------------------------------------------------------------------
// Entangler decomposition.  A rank-<=2 operator U = A_0 (x) B_0 + A_1 (x) B_1
// (found by rank-revealing elimination of the realigned 4x4) is brought to
// U = (A_0 V (x) I)[sum_a P_a (x) (B_0 + m_a B_1)](V^-1 (x) I) where
// A_0^-1 A_1 = V diag(m) V^-1.
int split_entangler(const cd* u, Split* s, std::string* err) {
  // realigned R[(a a')][(b b')] = U[2a+b][2a'+b']
  cd R[4][4];
  for (int a = 0; a < 2; ++a)
    for (int ap = 0; ap < 2; ++ap)
      for (int b = 0; b < 2; ++b)
        for (int bp = 0; bp < 2; ++bp) R[2 * a + ap][2 * b + bp] = u[4 * (2 * a + b) + (2 * ap + bp)];
  double scale = 0;
  for (auto& row : R)
    for (auto& v : row) scale = std::max(scale, std::abs(v));
  if (scale == 0) return fail(err, kErrRank, "entangler is the zero operator");
  const double tol = 1e-10 * scale;
  cd col[2][4], rowv[2][4];
  int rank = 0;
  cd W[4][4];
  std::memcpy(W, R, sizeof(W));
  for (int step = 0; step < 3; ++step) {
    int pi = 0, pj = 0;
    double best = -1;
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j)
        if (std::abs(W[i][j]) > best) { best = std::abs(W[i][j]); pi = i; pj = j; }
    if (best <= tol) break;
    if (step == 2) return fail(err, kErrRank, "entangler has operator Schmidt rank > 2");
    cd piv = W[pi][pj];
    for (int i = 0; i < 4; ++i) { col[step][i] = W[i][pj]; rowv[step][i] = W[pi][i] / piv; }
    for (int i = 0; i < 4; ++i)
      for (int j = 0; j < 4; ++j) W[i][j] -= col[step][i] * rowv[step][j];
    rank = step + 1;
  }
  M2 A[2], B[2];
  for (int t = 0; t < 2; ++t) {
    A[t] = M2::zero();
    B[t] = M2::zero();
  }
  for (int t = 0; t < rank; ++t)
    for (int i = 0; i < 4; ++i) { A[t].a[i] = col[t][i]; B[t].a[i] = rowv[t][i]; }
  // make A_0 invertible by re-mixing the Schmidt pair
  if (std::abs(det2(A[0])) < 1e-9 * std::max(1e-300, std::norm(A[0].a[0]) + std::norm(A[0].a[1]) +
                                                        std::norm(A[0].a[2]) + std::norm(A[0].a[3]))) {
    const cd ts[] = {cd(1), cd(-1), cd(0, 1), cd(2), cd(0, -2), cd(0.5, 0.5)};
    double bestd = -1;
    cd bt = 0;
    for (cd t : ts) {
      double dd = std::abs(det2(add(A[0], A[1], t)));
      if (dd > bestd) { bestd = dd; bt = t; }
    }
    if (bestd < 1e-12 * scale * scale) return fail(err, kErrRank, "entangler has no copy form (singular Schmidt factors)");
    A[0] = add(A[0], A[1], bt);
    B[1] = add(B[1], B[0], -bt);
  }
  M2 Mm = inverse(A[0]) * A[1];
  cd tr = Mm.a[0] + Mm.a[3], dt = det2(Mm);
  cd disc = std::sqrt(tr * tr - 4.0 * dt);
  cd lam[2] = {(tr + disc) / 2.0, (tr - disc) / 2.0};
  M2 V;
  double mscale = std::max(1.0, maxabs(Mm.a, 4));
  if (std::abs(lam[0] - lam[1]) > 1e-8 * mscale) {
    for (int e = 0; e < 2; ++e) {
      cd v1[2] = {Mm(0, 1), lam[e] - Mm(0, 0)};
      cd v2[2] = {lam[e] - Mm(1, 1), Mm(1, 0)};
      double n1 = std::norm(v1[0]) + std::norm(v1[1]), n2 = std::norm(v2[0]) + std::norm(v2[1]);
      const cd* v = n1 >= n2 ? v1 : v2;
      double nn = std::sqrt(std::max(n1, n2));
      V(0, e) = v[0] / nn;
      V(1, e) = v[1] / nn;
    }
  } else {
    if (std::abs(Mm(0, 1)) > 1e-8 * mscale || std::abs(Mm(1, 0)) > 1e-8 * mscale ||
        std::abs(Mm(0, 0) - Mm(1, 1)) > 1e-8 * mscale)
      return fail(err, kErrRank, "entangler has no copy form (defective Schmidt pencil)");
    V = M2();
  }
  s->pre = inverse(V);
  s->post = A[0] * V;
  s->C[0] = add(B[0], B[1], lam[0]);
  s->C[1] = add(B[0], B[1], lam[1]);
  // verify the reconstruction
  double worst = 0;
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      for (int ap = 0; ap < 2; ++ap)
        for (int bp = 0; bp < 2; ++bp) {
          cd acc = 0;
          for (int al = 0; al < 2; ++al) acc += s->post(a, al) * s->pre(al, ap) * s->C[al](b, bp);
          worst = std::max(worst, std::abs(acc - u[4 * (2 * a + b) + (2 * ap + bp)]));
        }
  if (worst > 1e-8 * scale) return fail(err, kErrRank, "entangler decomposition failed to reconstruct");
  return 0;
}

namespace {

Split cz_split() {
  Split s;
  s.C[0] = M2();
  s.C[1] = diag(1.0, -1.0);
  return s;
}

struct Event {
  int layer;
  bool up;  // true: consumes a slot of cut r-1 (row r is the lower qubit)
  int slot;
  const Split* sp;
};

struct RowChain {
  std::vector<Event> ev;
  cd v[2];              // start vector entering e_1
  std::vector<M2> seg;  // seg[i] between ev[i] and ev[i+1]  (size M-1)
  cd f[2][2];           // end row vector after ev[M-1], per output bit
};

int pair_index(const Plan& p, int layer, int cut) { return (layer - 1) * (p.n - 1) + cut; }

bool in_pattern(const Plan& p, int layer, int cut) {
  return ((p.parity1 + layer - 1) & 1) == (cut & 1);
}

// product L_{b-1} ... L_a on row r (identity when a == b)
M2 prod1q(const Plan& p, int r, int a, int b) {
  M2 m;
  for (int l = a; l < b; ++l) m = p.one[(size_t)l * p.n + r] * m;
  return m;
}

RowChain build_chain(const Plan& p, int r) {
  RowChain rc;
  for (int l = 1; l <= p.d; ++l) {
    if (r >= 1 && in_pattern(p, l, r - 1)) {
      const auto& X = p.X[r - 1];
      int s = int(std::lower_bound(X.begin(), X.end(), l) - X.begin());
      rc.ev.push_back({l, true, s, &p.split[pair_index(p, l, r - 1)]});
    } else if (r <= p.n - 2 && in_pattern(p, l, r)) {
      const auto& X = p.X[r];
      int s = int(std::lower_bound(X.begin(), X.end(), l) - X.begin());
      rc.ev.push_back({l, false, s, &p.split[pair_index(p, l, r)]});
    }
  }
  const int M = int(rc.ev.size());
  // start vector
  {
    M2 m = prod1q(p, r, 0, rc.ev[0].layer);
    if (!rc.ev[0].up) m = rc.ev[0].sp->pre * m;
    rc.v[0] = m(0, 0);
    rc.v[1] = m(1, 0);
  }
  for (int i = 0; i + 1 < M; ++i) {
    M2 m = prod1q(p, r, rc.ev[i].layer, rc.ev[i + 1].layer);
    if (!rc.ev[i].up) m = m * rc.ev[i].sp->post;
    if (!rc.ev[i + 1].up) m = rc.ev[i + 1].sp->pre * m;
    rc.seg.push_back(m);
  }
  {
    M2 m = prod1q(p, r, rc.ev[M - 1].layer, p.d + 1);
    if (!rc.ev[M - 1].up) m = m * rc.ev[M - 1].sp->post;
    for (int x = 0; x < 2; ++x) {
      rc.f[x][0] = m(x, 0);
      rc.f[x][1] = m(x, 1);
    }
  }
  return rc;
}

// K[alpha][beta] = (Lm * C_beta * Rm)[rowsel][colsel] variants
// a_of: function giving the matrix for (control a): returns M2 over (alpha, beta)
SweepOp make_op(int target, int control, int row) {
  SweepOp op;
  op.target = target;
  op.control = control;
  op.row = row;
  for (auto& v : op.mat)
    for (auto& m : v) m = M2::zero();
  return op;
}

// Ops of middle row r.
int build_row_ops(const Plan& p, int r, std::vector<SweepOp>* ops, int* ascending, std::string* err) {
  RowChain rc = build_chain(p, r);
  const auto& ev = rc.ev;
  const int M = int(ev.size());
  // events must alternate up/down
  for (int i = 0; i + 1 < M; ++i)
    if (ev[i].up == ev[i + 1].up) return fail(err, kErrInvalid, "row events do not alternate");
  if (M < 2) return fail(err, kErrInvalid, "middle row with fewer than two events");
  ops->clear();
  if (ev[0].up) {
    *ascending = 1;
    // pairs (ev[2j] up, ev[2j+1] down)
    int npairs = M / 2;
    for (int j = 0; j < npairs; ++j) {
      const Event& up = ev[2 * j];
      const Event& dn = ev[2 * j + 1];
      if (up.slot != j || dn.slot != j) return fail(err, kErrInvalid, "slot schedule mismatch (asc)");
      SweepOp op = make_op(j, j == 0 ? -1 : j - 1, r);
      for (int a = 0; a < (j == 0 ? 1 : 2); ++a) {
        for (int beta = 0; beta < 2; ++beta) {
          cd in[2];
          if (j == 0) {
            in[0] = rc.v[0];
            in[1] = rc.v[1];
          } else {
            in[0] = rc.seg[2 * j - 1](0, a);
            in[1] = rc.seg[2 * j - 1](1, a);
          }
          cd t1[2], t2[2];
          mat_vec(up.sp->C[beta], in, t1);
          mat_vec(rc.seg[2 * j], t1, t2);
          for (int al = 0; al < 2; ++al) op.mat[0][a](al, beta) = t2[al];
        }
      }
      if (j == 0) op.mat[0][1] = op.mat[0][0];
      ops->push_back(op);
    }
    if (M % 2 == 0) {
      // ends with a down event: scale rows by f_x
      SweepOp& last = ops->back();
      last.xrow[0] = r;
      const M2 base[2] = {last.mat[0][0], last.mat[0][1]};
      for (int x = 0; x < 2; ++x)
        for (int a = 0; a < 2; ++a) {
          M2 m = base[a];
          for (int al = 0; al < 2; ++al)
            for (int be = 0; be < 2; ++be) m(al, be) *= rc.f[x][al];
          last.mat[2 * x][a] = m;
        }
    } else {
      // ends with an up event in slot J: remove it, controlled by slot J-1
      int J = M / 2;
      const Event& up = ev[M - 1];
      if (up.slot != J || J < 1) return fail(err, kErrInvalid, "slot schedule mismatch (remove)");
      SweepOp op = make_op(J, J - 1, r);
      op.xrow[0] = r;
      for (int x = 0; x < 2; ++x)
        for (int a = 0; a < 2; ++a)
          for (int beta = 0; beta < 2; ++beta) {
            cd t1[2], t2[2];
            rowvec_mul(rc.f[x], up.sp->C[beta], t1);
            rowvec_mul(t1, rc.seg[M - 2], t2);
            op.mat[2 * x][a](0, beta) = t2[a];
            op.mat[2 * x][a](1, beta) = 0;
          }
      ops->push_back(op);
    }
  } else {
    *ascending = 0;
    int idx = M - 1;  // walk backward in time
    bool first = true;
    if (!ev[M - 1].up) {
      // odd-depth turn: expand a new top slot (the last down event)
      int J = M / 2;  // M = 2J+1
      const Event& dtop = ev[M - 1];
      if (dtop.slot != J) return fail(err, kErrInvalid, "slot schedule mismatch (expand)");
      SweepOp dup = make_op(J, -1, r);
      dup.kind = OP_DUP;
      ops->push_back(dup);
      const Event& up = ev[M - 2];
      const Event& dn = ev[M - 3];
      if (up.slot != J - 1 || dn.slot != J - 1) return fail(err, kErrInvalid, "slot schedule mismatch (expand pair)");
      SweepOp op = make_op(J - 1, J, r);
      op.xrow[0] = r;
      for (int x = 0; x < 2; ++x)
        for (int a = 0; a < 2; ++a) {
          M2 K = rc.seg[M - 2] * up.sp->C[0];  // placeholder, overwritten below
          for (int beta = 0; beta < 2; ++beta) {
            M2 prod = rc.seg[M - 2] * up.sp->C[beta] * rc.seg[M - 3];
            for (int al = 0; al < 2; ++al) op.mat[2 * x][a](al, beta) = rc.f[x][a] * prod(a, al);
          }
          (void)K;
        }
      ops->push_back(op);
      idx = M - 4;
      first = false;
    }
    // remaining pairs (ev[idx] up, ev[idx-1] down), idx odd, going down
    for (; idx >= 1; idx -= 2) {
      const Event& up = ev[idx];
      const Event& dn = ev[idx - 1];
      int j = up.slot;
      if (dn.slot != j || !up.up || dn.up) return fail(err, kErrInvalid, "slot schedule mismatch (desc)");
      if (first) {
        SweepOp op = make_op(j, -1, r);
        op.xrow[0] = r;
        for (int x = 0; x < 2; ++x)
          for (int beta = 0; beta < 2; ++beta) {
            cd t1[2], t2[2];
            rowvec_mul(rc.f[x], up.sp->C[beta], t1);
            rowvec_mul(t1, rc.seg[idx - 1], t2);
            for (int al = 0; al < 2; ++al) op.mat[2 * x][0](al, beta) = t2[al];
            op.mat[2 * x][1] = op.mat[2 * x][0];
          }
        ops->push_back(op);
        first = false;
      } else {
        SweepOp op = make_op(j, j + 1, r);
        for (int a = 0; a < 2; ++a)
          for (int beta = 0; beta < 2; ++beta) {
            M2 prod = rc.seg[idx] * up.sp->C[beta] * rc.seg[idx - 1];
            for (int al = 0; al < 2; ++al) op.mat[0][a](al, beta) = prod(a, al);
          }
        ops->push_back(op);
      }
    }
    if (idx != -1) return fail(err, kErrInvalid, "descending row pairing mismatch");
    // multiply the last op's output rows by the start vector v
    SweepOp& last = ops->back();
    for (int var = 0; var < 4; ++var)
      for (int a = 0; a < 2; ++a)
        for (int al = 0; al < 2; ++al)
          for (int be = 0; be < 2; ++be) last.mat[var][a](al, be) *= rc.v[al];
  }
  // replicate unused variants
  for (auto& op : *ops) {
    if (op.kind != OP_CU) continue;
    if (op.xrow[0] < 0) op.mat[2][0] = op.mat[0][0], op.mat[2][1] = op.mat[0][1];
    op.mat[1][0] = op.mat[0][0];
    op.mat[1][1] = op.mat[0][1];
    op.mat[3][0] = op.mat[2][0];
    op.mat[3][1] = op.mat[2][1];
  }
  return 0;
}

// Merge B (a no-control CU on A's target) into A: result = B * A.
SweepOp merge_ops(const SweepOp& A, const SweepOp& B) {
  SweepOp r = A;
  int xa = A.xrow[0], xb = B.xrow[0];
  r.xrow[0] = xa;
  r.xrow[1] = xb;
  for (int x0 = 0; x0 < 2; ++x0)
    for (int x1 = 0; x1 < 2; ++x1) {
      int var = 2 * x0 + x1;
      for (int a = 0; a < 2; ++a) r.mat[var][a] = B.mat[2 * x1][0] * A.mat[2 * x0][a];
    }
  return r;
}

}  // namespace

// ---------------------------------------------------------------------------
int build_plan(int n, int d, const cd* one_qubit, int n_gate2, const Gate2In* gates,
               const Options& opt, std::unique_ptr<Plan>* out, std::string* err) {
  if (n < 2 || d < 2) return fail(err, kErrDomain, "need n >= 2 qubits and d >= 2 layers");
  if (n > 4096 || d > 4096) return fail(err, kErrDomain, "n or d too large");
  if (opt.bond != 0 && opt.bond != 2 && opt.bond != 4) return fail(err, kErrInvalid, "bond must be 0, 2 or 4");
  bool rank4 = opt.bond == 4;
  auto p = std::make_unique<Plan>();
  p->n = n;
  p->d = d;
  p->opt = opt;
  p->one.resize((size_t)(d + 1) * n);
  for (size_t i = 0; i < p->one.size(); ++i)
    for (int e = 0; e < 4; ++e) p->one[i].a[e] = one_qubit[4 * i + e];
  // brickwork parity from the first gate
  p->parity1 = 1;
  if (n_gate2 > 0) p->parity1 = ((gates[0].q - (gates[0].layer - 1)) % 2 + 2) % 2;
  p->split.assign((size_t)d * (n - 1), Split());
  p->g4.assign((size_t)d * (n - 1), std::vector<cd>());
  std::vector<char> seen((size_t)d * (n - 1), 0);
  const Split idsplit;  // identity entangler: C_0 = C_1 = I
  Split identity;
  identity.C[0] = M2();
  identity.C[1] = M2();
  for (int i = 0; i < n_gate2; ++i) {
    const Gate2In& g = gates[i];
    if (g.layer < 1 || g.layer > d || g.q < 0 || g.q > n - 2)
      return fail(err, kErrInvalid, "gate out of range");
    if (!in_pattern(*p, g.layer, g.q))
      return fail(err, kErrInvalid, "gate breaks the alternating brickwork pattern");
    size_t pi = (size_t)pair_index(*p, g.layer, g.q);
    if (seen[pi]) return fail(err, kErrInvalid, "duplicate gate on a pair in one layer");
    seen[pi] = 1;
    std::vector<cd> m16(16, cd(0));
    if (g.kind == 0) {
      p->split[pi] = cz_split();
      m16[0] = m16[5] = m16[10] = 1;
      m16[15] = -1;
    } else if (g.kind == 1) {
      for (int e = 0; e < 16; ++e) m16[e] = g.m[e];
      if (opt.bond != 4) {
        std::string why;
        int rc = split_entangler(g.m, &p->split[pi], &why);
        if (rc == kErrRank && opt.bond == 0) {
          rank4 = true;  // lowered with bond dimension four below
        } else if (rc) {
          if (err) *err = why;
          return rc;
        }
      }
    } else {
      return fail(err, kErrInvalid, "unknown gate kind");
    }
    p->g4[pi] = m16;
  }
  for (int l = 1; l <= d; ++l)
    for (int c = 0; c < n - 1; ++c) {
      size_t pi = (size_t)pair_index(*p, l, c);
      if (in_pattern(*p, l, c) && !seen[pi]) {
        p->split[pi] = identity;
        std::vector<cd> m16(16, cd(0));
        m16[0] = m16[5] = m16[10] = m16[15] = 1;
        p->g4[pi] = m16;
      }
    }
  (void)idsplit;
  p->X.assign(n - 1, {});
  p->h = 0;
  for (int c = 0; c < n - 1; ++c) {
    for (int l = 1; l <= d; ++l)
      if (in_pattern(*p, l, c)) p->X[c].push_back(l);
    p->h = std::max(p->h, int(p->X[c].size()));
  }
  if (rank4) {
    // operator Schmidt rank 4: two legs per crossing (plan4.cpp)
    int rc = build_rows4(*p, err);
    if (rc) return rc;
    *out = std::move(p);
    return 0;
  }
  if (p->h > 40) return fail(err, kErrDomain, "width above 40 is not supported");
  // row 0 build-up
  {
    RowChain rc = build_chain(*p, 0);
    p->m0 = int(rc.ev.size());
    for (auto& e : rc.ev)
      if (e.up) return fail(err, kErrInvalid, "row 0 has an up event");
    p->init_v[0] = rc.v[0];
    p->init_v[1] = rc.v[1];
    p->init_seg = rc.seg;
    for (int x = 0; x < 2; ++x)
      for (int a = 0; a < 2; ++a) p->init_f[x][a] = rc.f[x][a];
  }
  p->row_ops.assign(n, {});
  p->row_ascending.assign(n, 0);
  for (int r = 1; r <= n - 2; ++r) {
    int asc = 0;
    int rc = build_row_ops(*p, r, &p->row_ops[r], &asc, err);
    if (rc) return rc;
    p->row_ascending[r] = asc;
  }
  *out = std::move(p);
  return 0;
}

// ---------------------------------------------------------------------------
namespace {

// Live slot count after rows 0..r (bond dimension four: every cut has
// d - 1 slots).
int live_after_row(const Plan& p, int r) { return p.chi == 4 ? p.h : int(p.X[r].size()); }

std::vector<Window> window_grid(const Plan& p, int hmax) {
  const int T = p.opt.max_tile_bits;
  const int C = p.opt.low_bits;
  std::vector<Window> ws;
  if (hmax <= T) {
    Window w;
    w.lo_bits = 0;
    w.win_lo = 0;
    w.win_len = hmax;
    ws.push_back(w);
    return ws;
  }
  // boundaries b_0 = 0 < b_1 < ... < b_m = hmax-1, windows [b_i, b_{i+1}]
  std::vector<int> b;
  b.push_back(0);
  int b1 = T - 1;              // bottom window [0, T-1], contiguous
  int top_lo = hmax - (T - C);  // top window [top_lo, hmax-1] with C low slots
  // The top window is a turn (two rows' updates meet there), bound by its
  // arithmetic: one slot fewer gives it a smaller tile (more resident
  // blocks per CU) and moves one update per row to the window below.  Taken
  // for windows of up to nine slots when the middle windows still need no
  // extra pass (measured at w = 33: top turn 35.1 -> 30.3 ms, 5.93 -> 5.81 s
  // per batch; wider windows over few low slots would lose the conflict-free
  // LDS placement of some phases).
  {
    const int span = T - C - 1;
    auto mids = [&](int tl) { return tl - b1 <= 0 ? 0 : (tl - b1 + span - 1) / span; };
    if (T - C <= 9 && top_lo > b1 && top_lo + 1 < hmax - 1 && span > 0 && mids(top_lo + 1) == mids(top_lo))
      ++top_lo;
  }
  if (top_lo <= b1) {
    b.push_back(b1);
    b.push_back(hmax - 1);
  } else {
    b.push_back(b1);
    int span = T - C - 1;  // middle window [b_i, b_i + span] has span+1 slots
    int gap = top_lo - b1;
    int nmid = (gap + span - 1) / span;
    for (int i = 1; i < nmid; ++i) b.push_back(b1 + (int)std::lround((double)gap * i / nmid));
    b.push_back(top_lo);
    b.push_back(hmax - 1);
  }
  for (size_t i = 0; i + 1 < b.size(); ++i) {
    Window w;
    if (b[i] == 0) {
      w.lo_bits = 0;
      w.win_lo = 0;
      w.win_len = b[i + 1] + 1;
    } else {
      w.lo_bits = C;
      w.win_lo = b[i];
      w.win_len = b[i + 1] - b[i] + 1;
    }
    ws.push_back(w);
  }
  return ws;
}

// Windows overlapping by `ov` slots: the contiguous bottom [0, T-1], then
// windows of T - C slots above C low slots, evenly spaced up to the top slot
// (the bond-four wavefront's updates span three slots, so its windows
// overlap by two: a unit at a boundary then lies wholly in one of them).
std::vector<Window> window_grid_overlap(const Plan& p, int hmax, int ov) {
  const int T = p.opt.max_tile_bits;
  const int C = p.opt.low_bits;
  std::vector<Window> ws;
  Window w;
  w.lo_bits = 0;
  w.win_lo = 0;
  w.win_len = std::min(hmax, T);
  ws.push_back(w);
  if (hmax <= T) return ws;
  const int L = T - C;
  const int S = T - ov, E = hmax - 1;
  if (L <= ov) return window_grid(p, hmax);
  const int m = std::max(1, (E - S + 1 - ov + (L - ov) - 1) / (L - ov));
  const int last = E - L + 1;
  for (int k = 0; k < m; ++k) {
    Window x;
    x.lo_bits = C;
    x.win_lo = m == 1 ? std::max(S, last) : S + (int)std::lround((double)(last - S) * k / (m - 1));
    x.win_len = std::min(L, hmax - x.win_lo);
    if (x.win_lo < C) {  // would overlap the low slots: fall back
      return window_grid(p, hmax);
    }
    ws.push_back(x);
  }
  // the top turn one slot shorter when the window below still overlaps it by
  // ov slots (as in window_grid)
  const size_t nw = ws.size();
  if (L <= 9 && nw >= 3 && ws[nw - 1].win_len == L && ws[nw - 1].win_lo + L - 1 == E &&
      ws[nw - 2].win_lo + ws[nw - 2].win_len - 1 >= ws[nw - 1].win_lo + ov) {
    ws[nw - 1].win_lo += 1;
    ws[nw - 1].win_len -= 1;
  }
  return ws;
}

// GF(2) span of lane slot directions (bit masks), one basis vector per
// leading bit.
struct Gf2Basis {
  uint32_t b[32] = {};
  uint32_t reduce(uint32_t x) const {
    for (int bit = 31; bit >= 0 && x; --bit)
      if ((x >> bit) & 1u) {
        if (!b[bit]) return x;
        x ^= b[bit];
      }
    return x;
  }
  bool independent(uint32_t x) const { return reduce(x) != 0u; }
  void add(uint32_t x) {
    x = reduce(x);
    for (int bit = 31; bit >= 0; --bit)
      if ((x >> bit) & 1u) {
        b[bit] = x;
        return;
      }
  }
};

// Thread-bit order of a register phase: the tile bits (ascending in `free`)
// that thread bits 0, 1, ... sit on.  The lanes of one bank cycle of an
// 8-byte LDS access are lanes 0..15 (or 0..31); they meet distinct slots when
// the slot directions (lane_slot_dir) of lane bits 0..3 are independent
// modulo 16 and those of lane bits 0..4 modulo 32.  So lane bits 0..3 take
// the first tile bits that keep both spans growing, lane bit 4 (unless pinned
// to tile bit pin4) the first one that adds a fifth direction, lane bit 5 is
// pin5 when given, and the remaining bits follow in increasing order.
std::vector<int> lane_order(std::vector<int> free_bits, int pin4, int pin5) {
  std::vector<int> order;
  Gf2Basis b16, b32;
  if (pin4 >= 0) b32.add(lane_slot_dir(pin4));
  auto take = [&](size_t i) {
    const int p = free_bits[i];
    free_bits.erase(free_bits.begin() + (long)i);
    b16.add(lane_slot_dir(p) & 15u);
    b32.add(lane_slot_dir(p));
    order.push_back(p);
  };
  for (int lane = 0; lane < 4 && !free_bits.empty(); ++lane) {
    size_t pick = free_bits.size();
    for (size_t i = 0; i < free_bits.size() && pick == free_bits.size(); ++i) {
      const uint32_t dv = lane_slot_dir(free_bits[i]);
      if (b16.independent(dv & 15u) && b32.independent(dv)) pick = i;
    }
    for (size_t i = 0; i < free_bits.size() && pick == free_bits.size(); ++i)
      if (b32.independent(lane_slot_dir(free_bits[i]))) pick = i;
    take(pick == free_bits.size() ? 0 : pick);
  }
  if (pin4 >= 0) {
    order.push_back(pin4);
  } else if (!free_bits.empty()) {
    size_t pick = 0;
    for (size_t i = 0; i < free_bits.size(); ++i)
      if (b32.independent(lane_slot_dir(free_bits[i]))) {
        pick = i;
        break;
      }
    take(pick);
  }
  if (pin5 >= 0) order.push_back(pin5);
  for (int p : free_bits) order.push_back(p);
  return order;
}

bool op_fits(const SweepOp& op, const Window& w) {
  if (!w.contains(op.target)) return false;
  if (op.control >= 0 && !w.contains(op.control)) return false;
  if (op.pair >= 0 && !w.contains(op.pair)) return false;
  return true;
}

// Fill a phase's register bits up to R with bits next to the targets, never
// op 0's control ctl0.
void pad_regs(std::vector<int>& regs, int ctl0, int T, int R) {
  auto usable = [&](int c) {
    return c >= 0 && c < T && c != ctl0 && std::find(regs.begin(), regs.end(), c) == regs.end();
  };
  for (int dist = 1; int(regs.size()) < R && dist <= T; ++dist)
    for (int base : std::vector<int>(regs)) {
      for (int c : {base + dist, base - dist}) {
        if (int(regs.size()) >= R) break;
        if (usable(c)) regs.push_back(c);
      }
    }
  for (int c = 0; int(regs.size()) < R && c < T; ++c)
    if (usable(c)) regs.push_back(c);
}

// Bank-cycle conflicts of a lane order: 2 if lanes 0..3 do not reach 16
// distinct slots, plus 1 if lanes 0..4 do not reach 32.
int lane_conflicts(const std::vector<int>& order) {
  Gf2Basis b16, b32;
  int r16 = 0, r32 = 0;
  for (size_t t = 0; t < order.size() && t < 5; ++t) {
    const uint32_t dv = lane_slot_dir(order[t]);
    if (t < 4 && b16.independent(dv & 15u)) {
      b16.add(dv & 15u);
      ++r16;
    }
    if (b32.independent(dv)) {
      b32.add(dv);
      ++r32;
    }
  }
  const int want16 = std::min<int>(4, (int)order.size()), want32 = std::min<int>(5, (int)order.size());
  return (r16 < want16 ? 2 : 0) + (r32 < want32 ? 1 : 0);
}

// The padding registers of a phase whose targets are `regs`: the bits next
// to the targets (pad_regs), unless another choice leaves free bits on which
// the lanes of a bank cycle meet distinct LDS slots (lane_order); candidates
// are tried nearest first.
void pad_regs_lds(std::vector<int>& regs, int ctl0, int T, int R) {
  std::vector<int> near = regs;
  pad_regs(near, ctl0, T, T);  // every usable bit, nearest first
  const std::vector<int> cand(near.begin() + (long)regs.size(), near.end());
  const int need = R - (int)regs.size();
  auto free_of = [&](const std::vector<int>& rg) {
    std::vector<int> f;
    for (int c = 0; c < T; ++c)
      if (std::find(rg.begin(), rg.end(), c) == rg.end()) f.push_back(c);
    return f;
  };
  std::vector<int> best = regs;
  pad_regs(best, ctl0, T, R);
  if (need <= 0 || T - R < 4) {
    regs = best;
    return;
  }
  int best_score = lane_conflicts(lane_order(free_of(best), -1, -1));
  if (best_score == 0 || need > (int)cand.size()) {
    regs = best;
    return;
  }
  // combinations of `need` candidates, lexicographic over the nearest-first list
  std::vector<int> idx(need);
  for (int q = 0; q < need; ++q) idx[q] = q;
  for (int tries = 0; tries < 4096; ++tries) {
    std::vector<int> rg = regs;
    for (int q : idx) rg.push_back(cand[q]);
    const int sc = lane_conflicts(lane_order(free_of(rg), -1, -1));
    if (sc < best_score) {
      best_score = sc;
      best = rg;
      if (sc == 0) break;
    }
    int q = need - 1;
    while (q >= 0 && idx[q] == (int)cand.size() - need + q) --q;
    if (q < 0) break;
    ++idx[q];
    for (int r = q + 1; r < need; ++r) idx[r] = idx[r - 1] + 1;
  }
  regs = best;
}

// The first three updates from op i can run as one fused product: plain
// updates with no output-bit variants.
bool fusable_start(const std::vector<SweepOp>& ops, int i, int end) {
  if (i + 3 > end) return false;
  for (int b = 0; b < 3; ++b) {
    const SweepOp& op = ops[i + b];
    if (op.kind != OP_CU || op.xrow[0] >= 0 || op.xrow[1] >= 0) return false;
  }
  return true;
}

// Register phases in canonical staircase form: op b of a phase targets
// register bit b and, for b >= 1, is controlled by register bit b-1; op 0 is
// either a DUP or an update whose control is not a register bit (or absent).
// Every row of the sweep is such a staircase; turns start a new phase.
// fuse: the phases will be given to split_triples.  A phase that it will
// fuse keeps two of its targets in lane bits, so its staircase may run two
// updates past the register bits (one when op 0's control takes the top
// register bit).
void plan_phases(Pass& ps, const std::vector<SweepOp>& ops, int R, bool fuse) {
  const int T = ps.w.tile_bits();
  const int Reff = pass_reg_bits(R, T);
  fuse = fuse && Reff >= 3 && T - Reff >= 6 && T - Reff <= kMaxThreadBits;
  // a bond-four wavefront step: 4x4s A on (a, a+1) and B on (a+1, a+2)
  // without output-bit variants
  auto unit_at = [&](int k) {
    if (k + 3 >= ps.op_end || ops[k].kind != OP_D4 || ops[k + 2].kind != OP_D4) return false;
    const SweepOp& A = ops[k];
    const SweepOp& B = ops[k + 2];
    return B.target == A.pair && B.pair == A.pair + 1 && A.pair == A.target + 1 && A.xrow[0] < 0 && A.xrow[1] < 0 &&
           B.xrow[0] < 0 && B.xrow[1] < 0;
  };
  int i = ps.op_begin;
  while (i < ps.op_end) {
    Phase ph;
    ph.op_begin = i;
    if (fuse && unit_at(i)) {
      // unit phase: A and B as one 8x8 on the matrix cores (b0 = register
      // bit 0, b1 and b2 = lane bits 4 and 5), then the next step (C on
      // (a-2, a-1), D on (a-1, a)) on register bits (1, 2) and (2, 0)
      const int b0 = ps.w.local(ops[i].target), b1 = ps.w.local(ops[i].pair), b2 = ps.w.local(ops[i + 2].pair);
      std::vector<int> regs = {b0};
      int j = i + 4;
      const int a = ops[i].target;
      if (i + 7 < ps.op_end && ops[i + 4].kind == OP_D4 && ops[i + 6].kind == OP_D4 && a >= 2 &&
          ops[i + 4].target == a - 2 && ops[i + 4].pair == a - 1 && ops[i + 6].target == a - 1 &&
          ops[i + 6].pair == a) {
        regs.push_back(ps.w.local(a - 2));
        regs.push_back(ps.w.local(a - 1));
        ph.dreg[2][0] = 1;
        ph.dreg[2][1] = 2;
        ph.dreg[3][0] = 2;
        ph.dreg[3][1] = 0;
        j = i + 8;
      }
      ph.op_end = j;
      ph.mf = 3;
      std::vector<int> rest;
      for (int c = 0; c < T; ++c)
        if (c != b1 && c != b2 && std::find(regs.begin(), regs.end(), c) == regs.end()) rest.push_back(c);
      const std::vector<int> lanes = lane_order(rest, b1, b2);
      for (int t = 0; t < 6; ++t) ph.tpos[t] = lanes[t];
      std::vector<int> left(lanes.begin() + 6, lanes.end());
      size_t q = 0;
      while (int(regs.size()) < Reff) regs.push_back(left[q++]);
      for (int r = 0; r < kMaxReg; ++r) ph.reg[r] = r < int(regs.size()) ? regs[r] : -1;
      const int TB = T - Reff;
      for (int t = 6; t < TB; ++t) ph.tpos[t] = left[q++];
      for (int t = TB; t < kMaxThreadBits; ++t) ph.tpos[t] = -1;
      ps.phases.push_back(ph);
      i = j;
      continue;
    }
    if (ops[i].kind == OP_D4) {
      // dense phase: up to four consecutive 4x4 updates whose slots fit in
      // the register bits (they may share slots: the updates run in order)
      std::vector<int> regs;
      auto at = [&](int b) { return int(std::find(regs.begin(), regs.end(), b) - regs.begin()); };
      int j = i, g = 0;
      while (j + 1 < ps.op_end && ops[j].kind == OP_D4 && g < 4) {
        const int lo = ps.w.local(ops[j].target), hi = ps.w.local(ops[j].pair);
        const int need = int(regs.size()) + (at(lo) == int(regs.size()) ? 1 : 0) + (at(hi) == int(regs.size()) ? 1 : 0);
        if (need > std::min(5, Reff)) break;
        if (at(lo) == int(regs.size())) regs.push_back(lo);
        if (at(hi) == int(regs.size())) regs.push_back(hi);
        ph.dreg[g][0] = at(lo);
        ph.dreg[g][1] = at(hi);
        j += 2;
        ++g;
      }
      // the longest prefix with a kernel form (one update always has one)
      while (g > 1) {
        uint32_t codes = 0;
        for (int q = 0; q < g; ++q)
          codes |= (uint32_t)dense_pair_code(std::min(ph.dreg[q][0], ph.dreg[q][1]),
                                             std::max(ph.dreg[q][0], ph.dreg[q][1])) << (4 * q);
        if (dense_form_exists(std::min(5, Reff), g, codes)) break;
        --g;
        j -= 2;
      }
      // registers of the dropped updates go back to padding
      {
        std::vector<int> keep;
        for (int q = 0; q < g; ++q)
          for (int b : {ph.dreg[q][0], ph.dreg[q][1]})
            if (std::find(keep.begin(), keep.end(), regs[b]) == keep.end()) keep.push_back(regs[b]);
        if (keep.size() < regs.size()) regs.resize(keep.size());  // a prefix: first-seen order
      }
      // (a tile too small for one dense update: the table builder refuses
      // the phase, which takes the update all the same)
      if (j == i) j = i + 2;
      ph.op_end = j;
      ph.mf = 2;
      pad_regs_lds(regs, -1, T, Reff);
      for (int q = 0; q < kMaxReg; ++q) ph.reg[q] = q < int(regs.size()) ? regs[q] : -1;
      std::vector<int> free_bits;
      for (int c = 0; c < T; ++c)
        if (std::find(regs.begin(), regs.end(), c) == regs.end()) free_bits.push_back(c);
      const std::vector<int> lanes = lane_order(free_bits, -1, -1);
      for (int t = 0; t < kMaxThreadBits; ++t) ph.tpos[t] = t < int(lanes.size()) ? lanes[t] : -1;
      ps.phases.push_back(ph);
      i = j;
      continue;
    }
    std::vector<int> regs = {ps.w.local(ops[i].target)};
    const int ctl0 = ops[i].kind == OP_CU && ops[i].control >= 0 ? ps.w.local(ops[i].control) : -1;
    const int limit = fuse && fusable_start(ops, i, ps.op_end) ? Reff + 2 - (ctl0 >= 0 ? 1 : 0) : Reff;
    int j = i + 1;
    for (; j < ps.op_end && int(regs.size()) < limit; ++j) {
      const SweepOp& op = ops[j];
      const int t = ps.w.local(op.target);
      if (op.kind != OP_CU || op.control < 0) break;
      if (ps.w.local(op.control) != regs.back()) break;
      if (std::find(regs.begin(), regs.end(), t) != regs.end() || t == ctl0) break;
      regs.push_back(t);
    }
    ph.op_end = j;
    pad_regs_lds(regs, ctl0, T, Reff);
    for (int q = 0; q < kMaxReg; ++q) ph.reg[q] = q < int(regs.size()) ? regs[q] : -1;
    std::vector<int> free_bits;
    for (int c = 0; c < T; ++c)
      if (std::find(regs.begin(), regs.end(), c) == regs.end()) free_bits.push_back(c);
    const std::vector<int> lanes = lane_order(free_bits, -1, -1);
    for (int t = 0; t < kMaxThreadBits; ++t) ph.tpos[t] = t < int(lanes.size()) ? lanes[t] : -1;
    ps.phases.push_back(ph);
    i = j;
  }
}

// Matrix-core phases (math = 2).  A staircase phase whose first three
// updates carry no output-bit variants runs those three as one fused 8x8
// product per value of op 0's control (targets b0 > register bit 0, b1, b2
// > lane bits 4, 5), then the rest of its staircase on the vector ALUs:
// update 3 targets register bit 1 under lane bit 5 (b2), update b > 3
// register bit b - 2 under register bit b - 3.  Op 0's control, if any, is
// the top register bit.  Needs six lane bits in the tile (T - R >= 6) and
// R >= 3.
void split_triples(Pass& ps, const std::vector<SweepOp>& ops) {
  const int T = ps.w.tile_bits();
  const int R = ps.R;
  const int TB = T - R;
  if (R < 3 || TB < 6 || TB > kMaxThreadBits) return;
  for (Phase& ph : ps.phases) {
    if (ph.mf == 2) continue;  // dense phases stay on the vector ALUs
    const int o = ph.op_begin;
    const int nops = ph.op_end - o;
    bool ok = nops >= 3;
    for (int b = 0; ok && b < 3; ++b) {
      const SweepOp& op = ops[o + b];
      if (op.kind != OP_CU || op.xrow[0] >= 0 || op.xrow[1] >= 0) ok = false;
    }
    if (!ok) continue;
    const int b0 = ph.reg[0], b1 = ph.reg[1], b2 = ph.reg[2];
    const int ctl0 = ops[o].control >= 0 ? ps.w.local(ops[o].control) : -1;
    std::vector<int> regs = {b0};
    for (int b = 3; b < nops; ++b) regs.push_back(ph.reg[b]);
    if (int(regs.size()) + (ctl0 >= 0 ? 1 : 0) > R) continue;
    auto used = [&](int c) {
      return c == b1 || c == b2 || c == ctl0 || std::find(regs.begin(), regs.end(), c) != regs.end();
    };
    std::vector<int> rest;
    for (int c = 0; c < T; ++c)
      if (!used(c)) rest.push_back(c);
    // lanes 0..3: free bits whose LDS slot directions keep the lanes of a
    // bank cycle apart (with b1 on lane 4), then the filler register bits,
    // then the wave bits
    Phase mp;
    mp.op_begin = o;
    mp.op_end = ph.op_end;
    mp.mf = 1;
    const std::vector<int> lanes = lane_order(rest, b1, b2);
    for (int t = 0; t < 6; ++t) mp.tpos[t] = lanes[t];
    std::vector<int> left(lanes.begin() + 6, lanes.end());
    size_t q = 0;
    while (int(regs.size()) < R - (ctl0 >= 0 ? 1 : 0)) regs.push_back(left[q++]);
    if (ctl0 >= 0) regs.push_back(ctl0);
    for (int r = 0; r < kMaxReg; ++r) mp.reg[r] = r < int(regs.size()) ? regs[r] : -1;
    for (int t = 6; t < TB; ++t) mp.tpos[t] = left[q++];
    for (int t = TB; t < kMaxThreadBits; ++t) mp.tpos[t] = -1;
    ph = mp;
  }
}

std::vector<Pass> plan_passes(const Plan& p, const std::vector<SweepOp>& ops, int R) {
  std::vector<Pass> passes;
  if (ops.empty()) return passes;
  auto ws = p.chi == 4 && !p.spatial ? window_grid_overlap(p, p.h, 2) : window_grid(p, p.h);
  int i = 0;
  const int nops = int(ops.size());
  while (i < nops) {
    // choose the window that contains the longest run of ops from i
    int best_w = -1, best_len = -1;
    for (int wi = 0; wi < int(ws.size()); ++wi) {
      int j = i;
      while (j < nops && op_fits(ops[j], ws[wi])) ++j;
      if (j - i > best_len) { best_len = j - i; best_w = wi; }
    }
    Pass ps;
    ps.w = ws[best_w];
    ps.op_begin = i;
    ps.op_end = i + best_len;
    const int T = ps.w.tile_bits();
    ps.R = pass_reg_bits(R, T);
    plan_phases(ps, ops, ps.R, p.opt.math == 2);
    // Fewer entries per thread leave registers for more resident waves:
    // take one register bit less when the pass needs no more phases with
    // it and a tile still fits one 256-thread block.
    if (p.opt.reg_adapt == 1 && ps.R >= 3 && T - (ps.R - 1) <= 8) {
      Pass alt = ps;
      alt.R = ps.R - 1;
      alt.phases.clear();
      plan_phases(alt, ops, alt.R, p.opt.math == 2);
      if (alt.phases.size() == ps.phases.size()) ps = alt;
    }
    if (p.opt.math == 2) split_triples(ps, ops);
    passes.push_back(ps);
    i += best_len;
  }
  return passes;
}

// Band evolution for Z_early: state of k qubits (bit j = qubit n-k+j).
void band_apply_u1(std::vector<cd>& st, int k, int bit, const M2& m) {
  const int dim = 1 << k;
  for (int i = 0; i < dim; ++i) {
    if (i >> bit & 1) continue;
    int i1 = i | (1 << bit);
    cd a0 = st[i], a1 = st[i1];
    st[i] = m(0, 0) * a0 + m(0, 1) * a1;
    st[i1] = m(1, 0) * a0 + m(1, 1) * a1;
  }
}

void band_apply_g4(std::vector<cd>& st, int k, int bit, const std::vector<cd>& g) {
  // bits (bit, bit+1) = (upper qubit, lower qubit); basis 2*x_upper + x_lower
  const int dim = 1 << k;
  for (int i = 0; i < dim; ++i) {
    if ((i >> bit & 1) || (i >> (bit + 1) & 1)) continue;
    int idx[4] = {i, i | (1 << (bit + 1)), i | (1 << bit), i | (1 << bit) | (1 << (bit + 1))};
    cd a[4], r[4];
    for (int u = 0; u < 4; ++u) a[u] = st[idx[u]];
    for (int o = 0; o < 4; ++o) {
      r[o] = 0;
      for (int u = 0; u < 4; ++u) r[o] += g[4 * o + u] * a[u];
    }
    for (int u = 0; u < 4; ++u) st[idx[u]] = r[u];
  }
}

double log2_sum(const std::vector<double>& log2s) {
  double mx = -1e300;
  for (double v : log2s) mx = std::max(mx, v);
  double s = 0;
  for (double v : log2s) s += std::exp2(v - mx);
  return mx + std::log2(s);
}

// Fold an end 2x2 `e` of a bond-dimension-four row (no control) into the
// dense 4x4 (halves a, b) listed just before it, on the slot e targets.
bool merge_into_dense(SweepOp& a, SweepOp& b, const SweepOp& e) {
  if (e.kind != OP_CU || e.control >= 0 || (e.target != a.target && e.target != a.pair)) return false;
  const bool ev = e.xrow[0] >= 0 || e.xrow[1] >= 0, dv = a.xrow[0] >= 0 || a.xrow[1] >= 0;
  if (ev && dv) return false;
  const int sh = e.target == a.target ? 0 : 1;
  for (int var = 0; var < 4; ++var) {
    cd M[4][4], R[4][4];
    for (int o = 0; o < 4; ++o)
      for (int u = 0; u < 4; ++u) M[o][u] = (o < 2 ? a : b).mat[var][o & 1].a[u];
    const M2& S = e.mat[var][0];
    for (int o = 0; o < 4; ++o)
      for (int u = 0; u < 4; ++u) {
        const int ob = (o >> sh) & 1;
        cd acc = 0;
        for (int t = 0; t < 2; ++t) acc += S(ob, t) * M[(o & ~(1 << sh)) | (t << sh)][u];
        R[o][u] = acc;
      }
    for (int o = 0; o < 4; ++o)
      for (int u = 0; u < 4; ++u) (o < 2 ? a : b).mat[var][o & 1].a[u] = R[o][u];
  }
  if (ev) {
    a.xrow[0] = b.xrow[0] = e.xrow[0];
    a.xrow[1] = b.xrow[1] = e.xrow[1];
  }
  return true;
}

// The schedule of a bond-dimension-four plan (k = 0): rows 1..n-2 as dense
// 4x4 updates, the end 2x2 of each row merged into the 4x4 before it, and
// the last row as the late program.
int schedule4(Plan& p, Schedule& s, std::string* err) {
  if (s.k != 0) return fail(err, kErrDomain, "open legs k >= 1 need entanglers of operator Schmidt rank <= 2");
  const int n = p.n, W = p.h;
  s.last_fixed_row = p.spatial ? n - 1 : n - 2;
  s.m_fix = W;
  auto emit = [&](const SweepOp& op) {
    const size_t m = s.ops.size();
    if (m >= 2 && s.ops[m - 2].kind == OP_D4 && merge_into_dense(s.ops[m - 2], s.ops[m - 1], op)) return;
    s.ops.push_back(op);
  };
  auto emit_gate = [&](const std::vector<SweepOp>& ro, size_t at) {
    emit(ro[at]);
    emit(ro[at + 1]);
  };
  if (p.spatial) {
    for (const SweepOp& op : p.row_ops[1]) emit(op);
  } else {
    // Rows go in pairs (A -> B row q, then B -> A row q+1), swept from the
    // top down as one wavefront: a 4x4 of row q+1 on (2j, 2j+1) follows
    // right after the 4x4 of row q on (2j-1, 2j), the last of its two
    // predecessors, so consecutive updates share slots and one pass carries
    // both rows through its window.  A row without a partner is listed on
    // its own.  Row q's 2x2 on slot 0 goes first (it meets nothing of row q
    // before row q+1's 4x4 on (0, 1)) and merges into the bottom 4x4 of the
    // pair before; row q+1's top 2x2 merges into row q's top 4x4.
    const int hc = (W + 1) / 2;
    int q = 1;
    while (q <= n - 2) {
      const std::vector<SweepOp>& A = p.row_ops[q];
      if (p.row_ascending[q] && q + 1 <= n - 2 && hc >= 2) {
        const std::vector<SweepOp>& B = p.row_ops[q + 1];
        // A: [2x2 on 0, 4x4 (2j-1, 2j) for j = 1..hc-1, two ops each]
        // B: [2x2 on top, 4x4 (2j, 2j+1) for j = hc-2..0, two ops each]
        auto a_at = [&](int j) { return (size_t)(1 + 2 * (j - 1)); };
        auto b_at = [&](int j) { return (size_t)(1 + 2 * (hc - 2 - j)); };
        emit(A[0]);
        emit_gate(A, a_at(hc - 1));
        emit(B[0]);
        for (int j = hc - 2; j >= 1; --j) {
          emit_gate(A, a_at(j));
          emit_gate(B, b_at(j));
        }
        emit_gate(B, b_at(0));
        q += 2;
      } else {
        for (const SweepOp& op : A) emit(op);
        q += 1;
      }
    }
  }
  // a dense update holds two register bits
  s.reg_bits = std::max(2, std::min(p.opt.reg_bits, W));
  s.passes = plan_passes(p, s.ops, s.reg_bits);
  int rc = build_late4(p, s, err);
  if (rc) return rc;
  // Cost in the |I||J||K| convention of Sec. 2.2: a crossing above absorbed
  // with its worldline piece costs 2^(W+3) (two steps of 2^(W+2)), the end
  // piece of a row 2^(W+1); build-up and the last row as for bond two.
  std::vector<double> cost;
  for (int j = 1; j <= p.m0; ++j) cost.push_back(j + 2.0);
  if (p.spatial) {
    // a two-qubit gate on the n-qubit state: 2^(n+2); a one-qubit gate 2^(n+1)
    for (const SweepOp& op : s.ops)
      if (op.kind != OP_D4H) cost.push_back(op.kind == OP_D4 ? W + 2.0 : W + 1.0);
  } else {
    const int hc = (W + 1) / 2;
    for (int r = 1; r <= n - 2; ++r) {
      for (int j = 0; j < hc - 1; ++j) cost.push_back(W + 3.0);
      cost.push_back(W + 1.0);
    }
  }
  for (int j = W; j >= 1; --j) cost.push_back(j + 1.0);
  s.log2_cost = log2_sum(cost);
  s.width = p.spatial ? n : W;
  return 0;
}

}  // namespace

int get_schedule(Plan& p, int k, std::shared_ptr<Schedule>* out, std::string* err) {
  if (k < 0 || k > p.n - 1) return fail(err, kErrDomain, "open legs k must satisfy 0 <= k <= n-1");
  if (k >= 1 && 2 * k > p.d) return fail(err, kErrDomain, "open legs k must satisfy 2k <= d");
  if (k > kMaxOpenLegs) return fail(err, kErrDomain, "open legs k above 10 are not supported");
  std::lock_guard<std::mutex> lk(p.mu);
  auto it = p.sched.find(k);
  if (it != p.sched.end()) {
    *out = it->second;
    return 0;
  }
  auto s = std::make_shared<Schedule>();
  s->k = k;
  const int n = p.n;
  if (p.chi == 4) {
    int rc = schedule4(p, *s, err);
    if (rc) return rc;
    p.sched[k] = s;
    *out = s;
    return 0;
  }
  s->last_fixed_row = (k == 0) ? n - 2 : n - k - 1;
  s->m_fix = live_after_row(p, s->last_fixed_row);
  // sweep ops: rows 1..last_fixed_row, merged at turns
  for (int r = 1; r <= s->last_fixed_row; ++r) {
    const auto& ro = p.row_ops[r];
    size_t start = 0;
    if (!s->ops.empty() && !ro.empty()) {
      SweepOp& prev = s->ops.back();
      const SweepOp& nx = ro[0];
      if (prev.kind == OP_CU && nx.kind == OP_CU && nx.control < 0 && nx.target == prev.target &&
          prev.xrow[1] < 0 && nx.xrow[1] < 0) {
        prev = merge_ops(prev, nx);
        start = 1;
      }
    }
    for (size_t i = start; i < ro.size(); ++i) s->ops.push_back(ro[i]);
  }
  s->reg_bits = std::max(1, std::min(p.opt.reg_bits, p.h));
  s->passes = plan_passes(p, s->ops, s->reg_bits);
  // late program
  const int d = p.d;
  std::vector<double> cost;
  if (k == 0) {
    s->s_bits = 1;
    s->join_u_bits = 0;
    RowChain rc = build_chain(p, n - 1);
    s->join = {rc.v[0], rc.v[1]};
    const int M = int(rc.ev.size());
    for (int j = 0; j < M; ++j) {
      if (!rc.ev[j].up || rc.ev[j].slot != j) return fail(err, kErrInvalid, "last row schedule mismatch");
      LateOp rm;
      rm.kind = L_REMOVE;
      for (int b = 0; b < 2; ++b)
        for (int e = 0; e < 4; ++e) rm.m.push_back(rc.ev[j].sp->C[b].a[e]);
      s->late.push_back(rm);
      if (j + 1 < M) {
        LateOp u;
        u.kind = L_U1;
        u.a = 0;
        for (int e = 0; e < 4; ++e) u.m.push_back(rc.seg[j].a[e]);
        s->late.push_back(u);
      }
    }
    LateOp dot;
    dot.kind = L_DOT;
    dot.xrow = n - 1;
    for (int x = 0; x < 2; ++x)
      for (int a = 0; a < 2; ++a) dot.m.push_back(rc.f[x][a]);
    s->late.push_back(dot);
    s->n_remove = M;
  } else {
    s->s_bits = k;
    s->join_u_bits = k;
    const int cut = n - k - 1;
    const auto& X = p.X[cut];
    const int c = 2 * k;
    if (int(X.size()) < k || X[k - 1] > c) return fail(err, kErrDomain, "fewer than k crossings in the early layers");
    const int dim = 1 << k;
    s->join.assign((size_t)dim * dim, cd(0));
    // One band state per assignment of the crossings met so far: states
    // branch at each crossing, so assignments share their common prefix
    // (u's bit j is the j-th crossing's index alpha).
    std::vector<std::vector<cd>> sts(1, std::vector<cd>(dim, cd(0)));
    sts[0][0] = 1;
    for (int l = 1; l <= c; ++l) {
      for (auto& st : sts) {
        for (int j = 0; j < k; ++j) band_apply_u1(st, k, j, p.one[(size_t)(l - 1) * n + (n - k + j)]);
        for (int j = 0; j + 1 < k; ++j) {
          int q = n - k + j;
          if (in_pattern(p, l, q)) band_apply_g4(st, k, j, p.g4[pair_index(p, l, q)]);
        }
      }
      if (in_pattern(p, l, cut)) {
        const int cj = int(std::lower_bound(X.begin(), X.end(), l) - X.begin());
        const Split& sp = p.split[pair_index(p, l, cut)];
        if (cj >= k) {
          for (auto& st : sts) band_apply_u1(st, k, 0, sp.C[0]);
        } else {
          // states are indexed by the bits of crossings 0..cj-1
          const size_t m = sts.size();
          if (m != (size_t)1 << cj) return fail(err, kErrInvalid, "early crossings out of order");
          sts.resize(2 * m);
          for (size_t i = 0; i < m; ++i) {
            sts[m + i] = sts[i];
            band_apply_u1(sts[i], k, 0, sp.C[0]);
            band_apply_u1(sts[m + i], k, 0, sp.C[1]);
          }
        }
      }
    }
    if ((int)sts.size() != dim) return fail(err, kErrInvalid, "early crossings do not match k");
    for (int u = 0; u < dim; ++u)
      for (int t = 0; t < dim; ++t) s->join[(size_t)u * dim + t] = sts[u][t];
    for (int l = c + 1; l <= d + 1; ++l) {
      for (int j = 0; j < k; ++j) {
        LateOp u1;
        u1.kind = L_U1;
        u1.a = j;
        const M2& g = p.one[(size_t)(l - 1) * n + (n - k + j)];
        for (int e = 0; e < 4; ++e) u1.m.push_back(g.a[e]);
        s->late.push_back(u1);
      }
      if (l > d) break;
      for (int j = 0; j + 1 < k; ++j) {
        int q = n - k + j;
        if (in_pattern(p, l, q)) {
          LateOp g4;
          g4.kind = L_G4;
          g4.a = j;
          g4.m = p.g4[pair_index(p, l, q)];
          s->late.push_back(g4);
        }
      }
      if (in_pattern(p, l, cut)) {
        LateOp rm;
        rm.kind = L_REMOVE;
        const Split& sp = p.split[pair_index(p, l, cut)];
        for (int b = 0; b < 2; ++b)
          for (int e = 0; e < 4; ++e) rm.m.push_back(sp.C[b].a[e]);
        s->late.push_back(rm);
        s->n_remove++;
      }
    }
    LateOp o;
    o.kind = L_OUT;
    s->late.push_back(o);
    if (s->n_remove != s->m_fix - k) return fail(err, kErrInvalid, "late removals do not match the live slots");
  }
  // Cost model in the |I||J||K| convention of Sec. 2.2: a paired update of
  // an R-leg boundary tensor costs 2^(R+2), a single absorption 2^(R+1).
  {
    int R = p.m0;
    for (int j = 1; j <= p.m0; ++j) cost.push_back(j + 2.0);  // row-0 build-up
    for (int r = 1; r <= s->last_fixed_row; ++r) {
      int rin = int(p.X[r - 1].size()), rout = int(p.X[r].size());
      R = std::max(rin, rout);
      // Alg. 1 on one row: the first tensor is absorbed alone (2^(R+1)),
      // then R-1 pairs (2^(R+2) each), then, when both cuts have R
      // crossings, the last tensor alone (2^(R+1)).
      for (int j = 0; j < R - 1; ++j) cost.push_back(R + 2.0);
      cost.push_back(R + 1.0);
      if (rin == rout) cost.push_back(R + 1.0);
    }
    R = s->m_fix;
    if (k == 0) {
      for (int j = R; j >= 1; --j) cost.push_back(j + 1.0);
    } else {
      cost.push_back(double(R + k));      // join: 2^(R-k) * 2^k * 2^k
      cost.push_back(2.0 * k + k + 2.0);  // early region (host)
      for (int j = R; j > k; --j) cost.push_back(j + 1.0);
    }
    s->log2_cost = log2_sum(cost);
    s->width = std::max(p.h, k >= 1 ? 2 * k : 0);
  }
  p.sched[k] = s;
  *out = s;
  return 0;
}

// ---------------------------------------------------------------------------
// FP64 host execution of the plan tables (self-check of the lowering).
namespace {

// Dense 4x4 (halves a, b) on the slot pair (a.target, a.pair).
void host_apply_dense(const SweepOp& a, const SweepOp& b, std::vector<cd>& B, int h, const uint8_t* x) {
  const size_t dim = size_t(1) << h;
  int var = 0;
  if (a.xrow[0] >= 0) var += 2 * x[a.xrow[0]];
  if (a.xrow[1] >= 0) var += x[a.xrow[1]];
  const size_t lo = size_t(1) << a.target, hi = size_t(1) << a.pair;
  for (size_t i = 0; i < dim; ++i) {
    if (i & (lo | hi)) continue;
    const size_t idx[4] = {i, i | lo, i | hi, i | lo | hi};
    cd in[4];
    for (int u = 0; u < 4; ++u) in[u] = B[idx[u]];
    for (int o = 0; o < 4; ++o) {
      const M2& row = (o < 2 ? a : b).mat[var][o & 1];
      cd acc = 0;
      for (int u = 0; u < 4; ++u) acc += row.a[u] * in[u];
      B[idx[o]] = acc;
    }
  }
}

void host_apply_op(const SweepOp& op, std::vector<cd>& B, int h, const uint8_t* x) {
  const size_t dim = size_t(1) << h;
  int var = 0;
  if (op.xrow[0] >= 0) var += 2 * x[op.xrow[0]];
  if (op.xrow[1] >= 0) var += x[op.xrow[1]];
  const size_t ts = size_t(1) << op.target;
  for (size_t i = 0; i < dim; ++i) {
    if (i & ts) continue;
    if (op.kind == OP_DUP) {
      B[i | ts] = B[i];
      continue;
    }
    int a = op.control >= 0 ? int((i >> op.control) & 1) : 0;
    const M2& m = op.mat[var][a];
    cd b0 = B[i], b1 = B[i | ts];
    B[i] = m(0, 0) * b0 + m(0, 1) * b1;
    B[i | ts] = m(1, 0) * b0 + m(1, 1) * b1;
  }
}

}  // namespace

int execute_host(Plan& p, int k, int n_batches, const uint8_t* bits, cd* out, std::string* err) {
  std::shared_ptr<Schedule> s;
  int rc = get_schedule(p, k, &s, err);
  if (rc) return rc;
  const int h = p.h, n = p.n;
  if (h > 24) return fail(err, kErrDomain, "host execution limited to width 24");
  const size_t dim = size_t(1) << h;
  for (int bt = 0; bt < n_batches; ++bt) {
    const uint8_t* x = bits + (size_t)bt * n;
    std::vector<cd> B(dim, cd(0));
    // row 0
    const int m0 = p.m0;
    for (size_t i = 0; i < (size_t(1) << m0); ++i) {
      cd v = p.init_v[i & 1];
      for (int j = 1; j < m0; ++j) v *= p.init_seg[j - 1](int(i >> j & 1), int(i >> (j - 1) & 1));
      v *= p.init_f[x[0]][int(i >> (m0 - 1) & 1)];
      B[i] = v;
    }
    for (size_t i = 0; i < s->ops.size(); ++i) {
      const SweepOp& op = s->ops[i];
      if (op.kind == OP_D4) host_apply_dense(op, s->ops[i + 1], B, h, x);
      else if (op.kind != OP_D4H) host_apply_op(op, B, h, x);
    }
    // late: state tensor st[rest][t] with t in the low s bits
    const int sb = s->s_bits;
    const int ub = s->join_u_bits;
    int rest_bits = s->m_fix - ub;
    std::vector<cd> st((size_t(1) << sb) << rest_bits, cd(0));
    const size_t sd = size_t(1) << sb;
    for (size_t rr = 0; rr < (size_t(1) << rest_bits); ++rr) {
      for (size_t t = 0; t < sd; ++t) {
        cd acc = 0;
        if (k == 0) {
          acc = s->join[t] * B[rr];
        } else {
          for (size_t u = 0; u < (size_t(1) << ub); ++u) acc += B[(rr << ub) | u] * s->join[u * sd + t];
        }
        st[(rr << sb) | t] = acc;
      }
    }
    cd* o = out + (size_t)bt * (size_t(1) << k);
    for (const auto& lo : s->late) {
      const size_t nrest = size_t(1) << rest_bits;
      if (lo.kind == L_U1) {
        M2 m;
        for (int e = 0; e < 4; ++e) m.a[e] = lo.m[e];
        for (size_t rr = 0; rr < nrest; ++rr) {
          std::vector<cd> v(st.begin() + rr * sd, st.begin() + (rr + 1) * sd);
          band_apply_u1(v, sb, lo.a, m);
          std::copy(v.begin(), v.end(), st.begin() + rr * sd);
        }
      } else if (lo.kind == L_G4) {
        for (size_t rr = 0; rr < nrest; ++rr) {
          std::vector<cd> v(st.begin() + rr * sd, st.begin() + (rr + 1) * sd);
          band_apply_g4(v, sb, lo.a, lo.m);
          std::copy(v.begin(), v.end(), st.begin() + rr * sd);
        }
      } else if (lo.kind == L_REMOVE || lo.kind == L_REMOVE2) {
        const int nb = lo.kind == L_REMOVE ? 1 : 2;
        const int off = (lo.kind == L_REMOVE && lo.xrow >= 0 && x[lo.xrow]) ? 8 : 0;
        M2 C[4];
        for (int b = 0; b < (1 << nb); ++b)
          for (int e = 0; e < 4; ++e) C[b].a[e] = lo.m[off + 4 * b + e];
        std::vector<cd> ns((sd << (rest_bits - nb)), cd(0));
        for (size_t rr = 0; rr < (nrest >> nb); ++rr)
          for (int u = 0; u < (1 << nb); ++u) {
            const size_t row = (rr << nb) | (size_t)u;
            std::vector<cd> v(st.begin() + row * sd, st.begin() + (row + 1) * sd);
            band_apply_u1(v, sb, 0, C[u]);
            for (size_t t = 0; t < sd; ++t) ns[rr * sd + t] += v[t];
          }
        st.swap(ns);
        rest_bits -= nb;
      } else if (lo.kind == L_DOT) {
        int xv = x[lo.xrow];
        o[0] = lo.m[2 * xv] * st[0] + lo.m[2 * xv + 1] * st[1];
      } else if (lo.kind == L_OUT) {
        for (size_t b = 0; b < sd; ++b) {
          size_t t = 0;
          for (int j = 0; j < k; ++j) t |= ((b >> (k - 1 - j)) & 1) << j;
          o[b] = st[t];
        }
      }
    }
    if (rest_bits != 0) return fail(err, kErrInvalid, "late program left slots");
  }
  return 0;
}

}  // namespace tnc
