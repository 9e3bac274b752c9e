// Bond-dimension-four lowering of the temporal-boundary contraction
// (Sec. 6.2, "Effect of bond dimension").
//
// Generic two-qubit gates reach operator Schmidt rank 4 (Sec. 2.1), so one
// binary copy index per crossing no longer carries it.  Written in matrix
// units of its upper qubit q, a gate on (q, q+1) is
//     G = sum_{a,b} |a><b| (x) U_ab,    U_ab[y'][y] = G[2a + y'][2b + y],
// and each crossing of cut (r|r+1) carries two binary legs: the value of the
// upper row's worldline entering the gate (`in`, b) and leaving it (`out`,
// a).  At even depth every cut has d/2 crossings and one of its legs is
// rank one:
//   type A (crossings at layers 1, 3, ..., d-1): `in` of the first crossing
//     is the upper row's start vector;
//   type B (crossings at layers 2, 4, ..., d): `out` of the last crossing
//     meets only the upper row's output functional.
// That leg is not stored: its vector (the start vector, or the output
// functional with its output-bit variant) is folded into the matrix of the
// update that consumes it one row later.  The boundary tensor thus has d-1
// binary slots, the constructive width min(n, d-1) of Sec. 6.2 for
// n >= d-1, in crossing order with the dropped leg left out:
//   type A: out_0, in_1, out_1, ..., in_{h-1}, out_{h-1}
//   type B: in_0, out_0, ..., in_{h-2}, out_{h-2}, in_{h-1}
// Absorbing a middle row maps the legs of the cut above onto those of the
// cut below along the row's worldline.  The worldline is cut open at each
// crossing below (its legs there are free indices), so the row factorises
// into one piece per crossing above, each joining that crossing's two legs
// to two legs of the cut below; at the same two slot positions, it is a
// dense 4x4 update on a slot pair (a 2x2 at one end of the row):
//   A -> B row ("ascending"):  2x2 on slot 0, then 4x4 on (2j-1, 2j);
//   B -> A row ("descending"): 2x2 on the top slot d-2 (with the output-bit
//     variants of the row above and of the row itself), 4x4 on (2j, 2j+1).
// The updates of one row act on disjoint slots and commute.  They are listed
// ascending in A -> B rows and descending in B -> A rows, so consecutive rows
// meet at the top or the bottom, where the end 2x2 of the next row is merged
// into the 4x4 before it (schedule assembly, plan.cpp).
//
// When n is below that width (n < d-1 at even depth, n <= d at odd depth)
// the narrower boundary is the spatial one: the n-qubit state, swept layer by
// layer (the constructive width min(n, d-1), resp. min(n, d), of Sec. 6.2).
// Its slots are the qubits; each layer is a set of dense 4x4 updates (the
// gate with the one-qubit layer after it) on the pattern pairs and 2x2s on
// the qubits outside them; the last layer also projects every qubit onto its
// output bit, (b_0, b_1) -> (b_x, 0), so that the tensor ends as the amplitude
// in entry 0 and zeros elsewhere, which the late program sums.
#include "plan.hpp"

#include <algorithm>
#include <cmath>

namespace tnc {

namespace {

constexpr int kErrInvalid = -1;
constexpr int kErrDomain = -2;

int fail4(std::string* err, int code, const std::string& msg) {
  if (err) *err = msg;
  return code;
}

int pair_at(const Plan& p, int layer, int cut) { return (layer - 1) * (p.n - 1) + cut; }

// Row r's one-qubit layers [a, b) in order: L_{b-1} ... L_a.
M2 layers(const Plan& p, int r, int a, int b) {
  M2 m;
  for (int l = a; l < b; ++l) m = p.one[(size_t)l * p.n + r] * m;
  return m;
}

// Lower-qubit block U_ab of the gate at (layer, cut).
M2 block(const Plan& p, int layer, int cut, int a, int b) {
  const std::vector<cd>& g = p.g4[pair_at(p, layer, cut)];
  M2 u;
  for (int yo = 0; yo < 2; ++yo)
    for (int yi = 0; yi < 2; ++yi) u(yo, yi) = g[4 * (2 * a + yo) + (2 * b + yi)];
  return u;
}

bool type_a(const Plan& p, int c) { return p.X[c][0] == 1; }

M2 add_scaled(const M2& x, cd a, const M2& y, cd b) {
  M2 r;
  for (int e = 0; e < 4; ++e) r.a[e] = a * x.a[e] + b * y.a[e];
  return r;
}

// Start vector of row r before layer l: its one-qubit layers 0..l-1 on |0>.
void start_vector(const Plan& p, int r, int l, cd v[2]) {
  const M2 m = layers(p, r, 0, l);
  v[0] = m(0, 0);
  v[1] = m(1, 0);
}

// Output functional of row r after layer l: f[x][w] = <x| L_d ... L_l |w>.
void end_functional(const Plan& p, int r, int l, cd f[2][2]) {
  const M2 m = layers(p, r, l, p.d + 1);
  for (int x = 0; x < 2; ++x)
    for (int w = 0; w < 2; ++w) f[x][w] = m(x, w);
}

SweepOp single_op(int target, int row) {
  SweepOp op;
  op.kind = OP_CU;
  op.target = target;
  op.control = -1;
  op.row = row;
  return op;
}

// The two halves of a dense 4x4 M (M[o][u], u = bit(lo) + 2 bit(hi)).
void push_dense(std::vector<SweepOp>* ops, int lo, int row, const cd M[4][4]) {
  for (int half = 0; half < 2; ++half) {
    SweepOp op;
    op.kind = half == 0 ? OP_D4 : OP_D4H;
    op.target = lo;
    op.pair = lo + 1;
    op.row = row;
    for (int var = 0; var < 4; ++var)
      for (int rr = 0; rr < 2; ++rr)
        for (int c = 0; c < 4; ++c) op.mat[var][rr].a[c] = M[2 * half + rr][c];
    ops->push_back(op);
  }
}

// Row q between a type-A cut r = q-1 above and a type-B cut q below.
void ascending_row(const Plan& p, int q, std::vector<SweepOp>* ops) {
  const int r = q - 1;
  const int hc = int(p.X[r].size());
  const std::vector<int>& Xa = p.X[r];  // 1, 3, ..., d-1
  const std::vector<int>& Xb = p.X[q];  // 2, 4, ..., d
  cd vr[2], vq[2];
  start_vector(p, r, Xa[0], vr);
  start_vector(p, q, Xa[0], vq);
  // slot 0 (out_0 above) -> in'_0 below:
  //   M[i'][o] = sum_in vr[in] (S U_{o,in} vq)[i'],  S = layers between the
  //   first crossing above and the first below
  {
    const M2 S = layers(p, q, Xa[0], Xb[0]);
    SweepOp op = single_op(0, q);
    M2 m = M2::zero();
    for (int o = 0; o < 2; ++o)
      for (int in = 0; in < 2; ++in) {
        const M2 K = S * block(p, Xa[0], r, o, in);
        for (int ip = 0; ip < 2; ++ip) m(ip, o) += vr[in] * (K(ip, 0) * vq[0] + K(ip, 1) * vq[1]);
      }
    for (auto& v : op.mat)
      for (auto& mm : v) mm = m;
    ops->push_back(op);
  }
  // crossing j >= 1 above (slots 2j-1 = in_j, 2j = out_j) -> out'_{j-1},
  // in'_j below (same slots): the worldline leaves crossing j-1 below as
  // out'_{j-1}, meets crossing j above, and enters crossing j below as in'_j
  for (int j = 1; j < hc; ++j) {
    const M2 Sa = layers(p, q, Xb[j - 1], Xa[j]);
    const M2 Sb = layers(p, q, Xa[j], Xb[j]);
    cd M[4][4];
    for (int in = 0; in < 2; ++in)
      for (int o = 0; o < 2; ++o) {
        const M2 K = Sb * block(p, Xa[j], r, o, in) * Sa;
        for (int op = 0; op < 2; ++op)
          for (int ip = 0; ip < 2; ++ip) M[op + 2 * ip][in + 2 * o] = K(ip, op);
      }
    push_dense(ops, 2 * j - 1, q, M);
  }
}

// Row q between a type-B cut r = q-1 above and a type-A cut q below.
void descending_row(const Plan& p, int q, std::vector<SweepOp>* ops) {
  const int r = q - 1;
  const int hc = int(p.X[r].size());
  const std::vector<int>& Xb = p.X[r];  // 2, 4, ..., d
  const std::vector<int>& Xa = p.X[q];  // 1, 3, ..., d-1
  const int top = 2 * hc - 2;
  // top slot (in_{h-1} above) -> out'_{h-1} below, variants (x_r, x_q):
  //   M[o'][in] = sum_out f_r[x_r][out] (f_q[x_q] U_{out,in} S)[o']
  {
    cd fr[2][2], fq[2][2];
    end_functional(p, r, Xb[hc - 1], fr);
    end_functional(p, q, Xb[hc - 1], fq);
    const M2 S = layers(p, q, Xa[hc - 1], Xb[hc - 1]);
    SweepOp op = single_op(top, q);
    op.xrow[0] = r;
    op.xrow[1] = q;
    for (int xr = 0; xr < 2; ++xr)
      for (int xq = 0; xq < 2; ++xq) {
        M2 m = M2::zero();
        for (int out = 0; out < 2; ++out)
          for (int in = 0; in < 2; ++in) {
            const M2 K = block(p, Xb[hc - 1], r, out, in) * S;
            for (int opr = 0; opr < 2; ++opr)
              m(opr, in) += fr[xr][out] * (fq[xq][0] * K(0, opr) + fq[xq][1] * K(1, opr));
          }
        op.mat[2 * xr + xq][0] = op.mat[2 * xr + xq][1] = m;
      }
    ops->push_back(op);
  }
  // crossing j <= h-2 above (slots 2j = in_j, 2j+1 = out_j) -> out'_j,
  // in'_{j+1} below: the worldline leaves crossing j below as out'_j, meets
  // crossing j above, and enters crossing j+1 below as in'_{j+1}
  for (int j = hc - 2; j >= 0; --j) {
    const M2 Sa = layers(p, q, Xa[j], Xb[j]);
    const M2 Sb = layers(p, q, Xb[j], Xa[j + 1]);
    cd M[4][4];
    for (int in = 0; in < 2; ++in)
      for (int o = 0; o < 2; ++o) {
        const M2 K = Sb * block(p, Xb[j], r, o, in) * Sa;
        for (int op = 0; op < 2; ++op)
          for (int ip = 0; ip < 2; ++ip) M[op + 2 * ip][in + 2 * o] = K(ip, op);
      }
    push_dense(ops, 2 * j, q, M);
  }
}

// Dense 4x4 of a gate on (q, q+1) followed by one-qubit gates a (on q) and
// b (on q+1), in the slot basis u = bit(q) + 2 bit(q+1) (the gate's own
// basis is 2 x_q + x_{q+1}).
void spatial_gate(const Plan& p, int layer, int q, const M2& a, const M2& b, cd M[4][4]) {
  const std::vector<cd>& g = p.g4[pair_at(p, layer, q)];
  auto sw = [](int u) { return ((u & 1) << 1) | (u >> 1); };
  for (int o = 0; o < 4; ++o)
    for (int u = 0; u < 4; ++u) {
      cd acc = 0;
      for (int t = 0; t < 4; ++t) acc += a(o & 1, t & 1) * b(o >> 1, t >> 1) * g[4 * sw(t) + sw(u)];
      M[o][u] = acc;
    }
}

// The projection of the last layer onto output bit x: (b_0, b_1) -> (b_x, 0).
M2 project(int x) {
  M2 m = M2::zero();
  m(0, x) = 1;
  return m;
}

int build_spatial4(Plan& p, std::string* err) {
  const int n = p.n, d = p.d;
  if (n > kMaxPlanWidth) return fail4(err, kErrDomain, "width above 69 is not supported");
  // at least three slots (a pass tile holds a dense update and a thread
  // bit): a two-qubit chain keeps a third slot that stays zero
  p.h = std::max(n, 3);
  p.chi = 4;
  p.spatial = true;
  // layer-0 product state: B0[a] = prod_q (L_0 |0>)_q[a_q]
  p.m0 = n;
  cd v[2];
  start_vector(p, 0, 1, v);
  p.init_v[0] = v[0];
  p.init_v[1] = v[1];
  p.init_seg.assign(n - 1, M2());
  for (int q = 1; q < n; ++q) {
    start_vector(p, q, 1, v);
    M2 s;
    s(0, 0) = s(0, 1) = v[0];
    s(1, 0) = s(1, 1) = v[1];
    p.init_seg[q - 1] = s;
  }
  for (int x = 0; x < 2; ++x) p.init_f[x][0] = p.init_f[x][1] = 1;
  // layers 1..d, ascending in odd layers and descending in even ones
  p.row_ops.assign(2, {});
  std::vector<SweepOp>& ops = p.row_ops[1];
  for (int l = 1; l <= d; ++l) {
    const bool last = l == d;
    std::vector<char> paired(n, 0);
    std::vector<std::vector<SweepOp>> items(n);  // per lowest slot
    for (int q = 0; q + 1 < n; ++q) {
      if (p.g4[pair_at(p, l, q)].empty()) continue;  // not a pattern pair of this layer
      paired[q] = paired[q + 1] = 1;
      const M2& a = p.one[(size_t)l * n + q];
      const M2& b = p.one[(size_t)l * n + q + 1];
      std::vector<SweepOp> two;
      for (int var = 0; var < 4; ++var) {
        const int xq = var >> 1, xq1 = var & 1;
        cd M[4][4];
        spatial_gate(p, l, q, last ? project(xq) * a : a, last ? project(xq1) * b : b, M);
        if (var == 0) {
          push_dense(&two, q, l, M);
          if (last) {
            two[0].xrow[0] = two[1].xrow[0] = q;
            two[0].xrow[1] = two[1].xrow[1] = q + 1;
          }
        }
        for (int half = 0; half < 2; ++half)
          for (int rr = 0; rr < 2; ++rr)
            for (int c = 0; c < 4; ++c) two[half].mat[var][rr].a[c] = M[2 * half + rr][c];
      }
      items[q] = two;
    }
    for (int q = 0; q < n; ++q) {
      if (paired[q]) continue;
      SweepOp op = single_op(q, l);
      const M2& a = p.one[(size_t)l * n + q];
      if (last) {
        op.xrow[0] = q;
        op.mat[0][0] = op.mat[0][1] = op.mat[1][0] = op.mat[1][1] = project(0) * a;
        op.mat[2][0] = op.mat[2][1] = op.mat[3][0] = op.mat[3][1] = project(1) * a;
      } else {
        for (auto& vv : op.mat)
          for (auto& mm : vv) mm = a;
      }
      items[q] = {op};
    }
    if (l % 2) {
      for (int q = 0; q < n; ++q)
        for (const SweepOp& o : items[q]) ops.push_back(o);
    } else {
      for (int q = n - 1; q >= 0; --q)
        for (const SweepOp& o : items[q]) ops.push_back(o);
    }
  }
  return 0;
}

}  // namespace

int build_rows4(Plan& p, std::string* err) {
  const int n = p.n, d = p.d;
  // the narrower of the two boundaries (Sec. 6.2: min(n, d-1) at even depth,
  // min(n, d) at odd depth; the temporal one is built for even depth)
  if (d % 2 ? n <= d : n < d - 1) return build_spatial4(p, err);
  if (d % 2) return fail4(err, kErrDomain, "bond dimension 4 at odd depth needs n <= d");
  const int hc = d / 2;
  for (int c = 0; c < n - 1; ++c)
    if (int(p.X[c].size()) != hc) return fail4(err, kErrInvalid, "cut without d/2 crossings");
  for (int c = 0; c + 1 < n - 1; ++c)
    if (type_a(p, c) == type_a(p, c + 1)) return fail4(err, kErrInvalid, "cut types do not alternate");
  const int W = 2 * hc - 1;
  if (W > kMaxPlanWidth) return fail4(err, kErrDomain, "width above 69 is not supported");
  p.h = W;
  p.chi = 4;
  // row 0: its worldline is cut open at each of its crossings, so B_0 is a
  // product over the pieces between consecutive crossings; written as the
  // chain of the build-up kernel (B0[a] = v[a_0] prod_j seg_j[a_j][a_{j-1}]
  // f_x[a_{W-1}]) with all-ones links between the two legs of one crossing
  const std::vector<int>& X0 = p.X[0];
  M2 ones;
  ones.a[0] = ones.a[1] = ones.a[2] = ones.a[3] = 1;
  p.m0 = W;
  p.init_seg.assign(std::max(0, W - 1), ones);
  if (type_a(p, 0)) {
    // slots out'_0, in'_1, out'_1, ...: the piece between crossings j and
    // j+1 links slot 2j (out'_j) to slot 2j+1 (in'_{j+1})
    p.init_v[0] = p.init_v[1] = 1;
    for (int j = 0; j + 1 < hc; ++j) p.init_seg[2 * j] = layers(p, 0, X0[j], X0[j + 1]);
    cd f[2][2];
    end_functional(p, 0, X0[hc - 1], f);
    for (int x = 0; x < 2; ++x)
      for (int a = 0; a < 2; ++a) p.init_f[x][a] = f[x][a];
  } else {
    // slots in'_0, out'_0, in'_1, ...: slot 2j+1 (out'_j) to 2j+2 (in'_{j+1})
    start_vector(p, 0, X0[0], p.init_v);
    for (int j = 0; j + 1 < hc; ++j) p.init_seg[2 * j + 1] = layers(p, 0, X0[j], X0[j + 1]);
    for (int x = 0; x < 2; ++x)
      for (int a = 0; a < 2; ++a) p.init_f[x][a] = 1;
  }
  p.row_ops.assign(n, {});
  p.row_ascending.assign(n, 0);
  for (int q = 1; q <= n - 2; ++q) {
    if (type_a(p, q - 1)) {
      ascending_row(p, q, &p.row_ops[q]);
      p.row_ascending[q] = 1;
    } else {
      descending_row(p, q, &p.row_ops[q]);
      p.row_ascending[q] = 0;
    }
  }
  return 0;
}

int build_late4(const Plan& p, Schedule& s, std::string* err) {
  const int n = p.n;
  if (p.spatial) {
    // the projected state: the amplitude in entry 0, zeros elsewhere; the
    // late program sums every entry (identity removals, then <0|)
    s.s_bits = 1;
    s.join_u_bits = 0;
    s.late.clear();
    s.n_remove = 0;
    s.join = {cd(1), cd(0)};
    for (int q = 0; q < p.h; ++q) {  // (the spare slot of n = 2 included)
      LateOp o;
      o.kind = L_REMOVE;
      const M2 id;
      for (int b = 0; b < 2; ++b)
        for (int e = 0; e < 4; ++e) o.m.push_back(id.a[e]);
      s.late.push_back(o);
      s.n_remove++;
    }
    LateOp dot;
    dot.kind = L_DOT;
    dot.xrow = 0;
    for (int x = 0; x < 2; ++x) {
      dot.m.push_back(cd(1));
      dot.m.push_back(cd(0));
    }
    s.late.push_back(dot);
    return 0;
  }
  const int c = n - 2, q = n - 1;
  const std::vector<int>& X = p.X[c];
  const int hc = int(X.size());
  s.s_bits = 1;
  s.join_u_bits = 0;
  s.late.clear();
  s.n_remove = 0;
  auto u1 = [&](const M2& m) {
    LateOp o;
    o.kind = L_U1;
    o.a = 0;
    for (int e = 0; e < 4; ++e) o.m.push_back(m.a[e]);
    s.late.push_back(o);
  };
  auto remove2 = [&](int layer) {
    LateOp o;
    o.kind = L_REMOVE2;
    for (int u = 0; u < 4; ++u) {
      const M2 b = block(p, layer, c, u >> 1, u & 1);  // u = in + 2 out
      for (int e = 0; e < 4; ++e) o.m.push_back(b.a[e]);
    }
    s.late.push_back(o);
    s.n_remove++;
  };
  cd v[2];
  start_vector(p, q, X[0], v);
  s.join = {v[0], v[1]};
  int removed = 0;
  if (type_a(p, c)) {
    // slot 0 is out_0; in_0 carries row c's start vector
    cd vc[2];
    start_vector(p, c, X[0], vc);
    LateOp o;
    o.kind = L_REMOVE;
    for (int b = 0; b < 2; ++b) {
      const M2 m = add_scaled(block(p, X[0], c, b, 0), vc[0], block(p, X[0], c, b, 1), vc[1]);
      for (int e = 0; e < 4; ++e) o.m.push_back(m.a[e]);
    }
    s.late.push_back(o);
    s.n_remove++;
    removed = 1;
    for (int j = 1; j < hc; ++j) {
      u1(layers(p, q, X[j - 1], X[j]));
      remove2(X[j]);
      removed += 2;
    }
  } else {
    // slots in_0, out_0, ..., in_{h-1}; out_{h-1} carries row c's output
    // functional (variant on x_c)
    for (int j = 0; j + 1 < hc; ++j) {
      if (j > 0) u1(layers(p, q, X[j - 1], X[j]));
      remove2(X[j]);
      removed += 2;
    }
    if (hc >= 2) u1(layers(p, q, X[hc - 2], X[hc - 1]));
    cd fc[2][2];
    end_functional(p, c, X[hc - 1], fc);
    LateOp o;
    o.kind = L_REMOVE;
    o.xrow = c;
    for (int x = 0; x < 2; ++x)
      for (int b = 0; b < 2; ++b) {
        const M2 m = add_scaled(block(p, X[hc - 1], c, 0, b), fc[x][0], block(p, X[hc - 1], c, 1, b), fc[x][1]);
        for (int e = 0; e < 4; ++e) o.m.push_back(m.a[e]);
      }
    s.late.push_back(o);
    s.n_remove++;
    removed += 1;
  }
  if (removed != p.h) return fail4(err, kErrInvalid, "last row does not remove every slot");
  cd f[2][2];
  end_functional(p, q, X[hc - 1], f);
  LateOp dot;
  dot.kind = L_DOT;
  dot.xrow = q;
  for (int x = 0; x < 2; ++x)
    for (int a = 0; a < 2; ++a) dot.m.push_back(f[x][a]);
  s.late.push_back(dot);
  return 0;
}

}  // namespace tnc
