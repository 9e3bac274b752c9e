// Late-phase launch construction (see late.hpp).
#include "late.hpp"

#include <algorithm>

namespace tnc {

namespace {

// cols[c * dim + t]: column c of a dim x dim operator, as a state vector.
void cols_u1(std::vector<cd>& cols, int sb, int bit, const cd* m) {
  const int dim = 1 << sb;
  for (int c = 0; c < dim; ++c) {
    cd* v = cols.data() + (size_t)c * dim;
    for (int i = 0; i < dim; ++i) {
      if (i >> bit & 1) continue;
      const int i1 = i | (1 << bit);
      const cd a0 = v[i], a1 = v[i1];
      v[i] = m[0] * a0 + m[1] * a1;
      v[i1] = m[2] * a0 + m[3] * a1;
    }
  }
}

void cols_g4(std::vector<cd>& cols, int sb, int bit, const cd* g) {
  const int dim = 1 << sb;
  for (int c = 0; c < dim; ++c) {
    cd* v = cols.data() + (size_t)c * dim;
    for (int i = 0; i < dim; ++i) {
      if ((i >> bit & 1) || (i >> (bit + 1) & 1)) continue;
      const int idx[4] = {i, i | (1 << (bit + 1)), i | (1 << bit), i | (1 << bit) | (1 << (bit + 1))};
      cd a[4], r[4];
      for (int u = 0; u < 4; ++u) a[u] = v[idx[u]];
      for (int o = 0; o < 4; ++o) {
        r[o] = 0;
        for (int u = 0; u < 4; ++u) r[o] += g[4 * o + u] * a[u];
      }
      for (int u = 0; u < 4; ++u) v[idx[u]] = r[u];
    }
  }
}

int bitrev(int b, int k) {
  int t = 0;
  for (int j = 0; j < k; ++j) t |= ((b >> (k - 1 - j)) & 1) << j;
  return t;
}

}  // namespace

int build_late(const Plan& p, const Schedule& s, LatePlan* out, std::string* err) {
  const auto& L = s.late;
  if (L.empty()) {
    if (err) *err = "empty late program";
    return -1;
  }
  const int sb = s.s_bits;
  const int dim = 1 << sb;
  const int k = s.k;
  out->s = sb;
  const LateOp& fin = L.back();
  out->final_kind = fin.kind;
  out->final_xrow = fin.xrow;
  if (fin.kind == L_DOT) out->dot = fin.m;
  const int nbody = int(L.size()) - 1;
  // removals and the slots they consume: slots_to[i] = slots removed by
  // removals 0..i-1
  std::vector<int> rpos, slots_to(1, 0);
  for (int i = 0; i < nbody; ++i)
    if (L[i].kind == L_REMOVE || L[i].kind == L_REMOVE2) {
      rpos.push_back(i);
      slots_to.push_back(slots_to.back() + (L[i].kind == L_REMOVE2 ? 2 : 1));
    }
  const int nrem = int(rpos.size());
  // k = 0: fold removals of up to 12 slots (the state is one qubit), but not
  // a removal with an output-bit variant (the first launch has one variant
  // row, the final one's).  k >= 1: folding j removals costs O(2^(3k+j)) on
  // the host and shrinks the first launch's FP64 output to 2^(m-j) rows;
  // worth it for large tensors only.  With no removal folded, the join
  // matrix is Z_early itself and every late op runs on the device.
  int j1;  // removals folded
  if (k == 0) {
    j1 = 0;
    while (j1 < nrem && slots_to[j1 + 1] <= 12 && L[rpos[j1]].xrow < 0) ++j1;
  } else {
    // 2^35-entry tensors (256 GiB of complex64) leave room for a join output
    // of 2^(h-j) x 16 B only with j = 7 (4 GiB; the fold takes ~4 s).  From
    // 2^30 entries on, j = 5 shrinks the late launches' input 32-fold for a
    // host fold of about a second; the join's flops do not depend on j.
    const int want = p.opt.late_fold == 0 ? (s.m_fix >= 35 ? 7 : s.m_fix >= 30 ? 5 : s.m_fix >= 26 ? 3 : 0)
                                          : std::max(0, p.opt.late_fold);
    j1 = std::min(nrem, std::min(want, k <= 8 ? 8 : 1));
  }
  const bool first_final = j1 == nrem;
  const int first_end = first_final ? nbody : (j1 == 0 ? 0 : rpos[j1 - 1] + 1);

  // P_u for each assignment u of the folded slots
  const int js = slots_to[j1];
  const int nu = 1 << js;
  std::vector<std::vector<cd>> P(nu);
  for (int u = 0; u < nu; ++u) {
    std::vector<cd> cols((size_t)dim * dim, cd(0));
    for (int c = 0; c < dim; ++c) cols[(size_t)c * dim + c] = 1;
    int l = 0;
    for (int i = 0; i < first_end; ++i) {
      const LateOp& o = L[i];
      if (o.kind == L_U1) cols_u1(cols, sb, o.a, o.m.data());
      else if (o.kind == L_G4) cols_g4(cols, sb, o.a, o.m.data());
      else if (o.kind == L_REMOVE) {
        const int b = (u >> l) & 1;
        cols_u1(cols, sb, 0, o.m.data() + 4 * b);
        ++l;
      } else if (o.kind == L_REMOVE2) {
        const int b = (u >> l) & 3;
        cols_u1(cols, sb, 0, o.m.data() + 4 * b);
        l += 2;
      }
    }
    P[u].swap(cols);
  }
  LateFirst& F = out->first;
  F.j = js;
  F.final = first_final;
  const int ub = s.join_u_bits;
  F.K = 1 << (ub + js);
  F.M = 1LL << (s.m_fix - ub - js);
  // unpermuted J: Ju[kk][t]
  std::vector<cd> Ju((size_t)F.K * dim, cd(0));
  for (int u = 0; u < nu; ++u) {
    const std::vector<cd>& cols = P[u];
    if (k == 0) {
      // kk = u; state entering = v (the join vector)
      for (int t = 0; t < dim; ++t) {
        cd acc = 0;
        for (int w = 0; w < dim; ++w) acc += cols[(size_t)w * dim + t] * s.join[w];
        Ju[(size_t)u * dim + t] = acc;
      }
    } else {
      const int de = 1 << ub;
      if (first_end == 0) {
        // nothing folded: P is the identity and J is the join matrix
        std::copy(s.join.begin(), s.join.begin() + (size_t)de * dim, Ju.begin() + ((size_t)u << ub) * dim);
        continue;
      }
      for (int ue = 0; ue < de; ++ue) {
        cd* row = Ju.data() + ((size_t)((u << ub) | ue)) * dim;
        for (int tp = 0; tp < dim; ++tp) {
          const cd z = s.join[(size_t)ue * dim + tp];
          if (z == cd(0)) continue;
          const cd* col = cols.data() + (size_t)tp * dim;
          for (int t = 0; t < dim; ++t) row[t] += z * col[t];
        }
      }
    }
  }
  if (!first_final) {
    F.N = dim;
    F.nvar = 1;
    F.xrow = -1;
    F.J.swap(Ju);
  } else if (fin.kind == L_OUT) {
    F.N = 1 << k;
    F.nvar = 1;
    F.J.assign((size_t)F.K * F.N, cd(0));
    for (int kk = 0; kk < F.K; ++kk)
      for (int b = 0; b < F.N; ++b) F.J[(size_t)kk * F.N + b] = Ju[(size_t)kk * dim + bitrev(b, k)];
  } else {
    F.N = 1;
    F.nvar = 2;
    F.xrow = fin.xrow;
    F.J.assign((size_t)2 * F.K, cd(0));
    for (int var = 0; var < 2; ++var)
      for (int kk = 0; kk < F.K; ++kk) {
        cd acc = 0;
        for (int t = 0; t < dim; ++t) acc += fin.m[2 * var + t] * Ju[(size_t)kk * dim + t];
        F.J[(size_t)var * F.K + kk] = acc;
      }
  }
  // remaining launches
  if (!first_final) {
    // each launch takes whole removals of at most jmax slots
    const int jmax = std::max(2, 12 - sb);
    int done = j1;
    int pos = first_end;
    long long rows = F.M;
    while (done < nrem) {
      int e = done + 1;
      while (e < nrem && slots_to[e + 1] - slots_to[done] <= jmax) ++e;
      const int j = slots_to[e] - slots_to[done];
      const bool last = e == nrem;
      const int end = last ? nbody : rpos[e - 1] + 1;
      LateOpsLaunch ln;
      ln.op_begin = pos;
      ln.op_end = end;
      ln.j = j;
      ln.rows_in = rows;
      ln.final = last;
      out->ops.push_back(ln);
      rows >>= j;
      done = e;
      pos = end;
    }
  }
  return 0;
}

}  // namespace tnc
