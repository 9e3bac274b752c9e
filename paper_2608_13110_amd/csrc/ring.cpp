// Ring geometry by structure-aware slicing (Sec. 6.3): the CZ gates of the
// wrap pair (n-1, 0) are cut, CZ = sum_a P_a (x) Z^a with P_a = |a><a| on
// qubit n-1 and Z^a on qubit 0.  Each of the 2^m assignments of the m cut
// bonds is an open-chain circuit (its P_a, Z^a factors folded into the
// one-qubit layer that follows the cut gate, where both qubits are idle in
// the chain pattern), planned and contracted like any other; the ring's
// amplitudes are the sum over the slices.  The slices share their shape
// (the same passes, phases and late program, other matrices), so they run
// in groups: the i-th launches of every slice of a group become one grouped
// launch (each slice a segment of its own arguments and workspace), as the
// server runs same-width requests together.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <complex>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/tnc.h"
#include "exec.hpp"
#include "kernels.hpp"

struct tnc_ring_plan_s {
  int n = 0, d = 0, m = 0;
  std::vector<tnc_plan_t> slices;
  // pinned staging of the grouped launches' segment tables, reused call to
  // call once the copy recorded by `copied` has completed
  unsigned char* h_seg = nullptr;
  size_t h_cap = 0;
  hipEvent_t copied = nullptr;
};

namespace {

int ring_err(int code, const std::string& msg) { return tnc::set_error_message(code, msg); }

uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

// Slices per group: every slice of a group holds its own workspace and
// result, so a group is bounded by 2 GiB of them (and by 1024 slices).
constexpr uint64_t kGroupBytes = 2ull << 30;
constexpr int kMaxGroup = 1024;
// Segment table bytes per slice and launch of a group.
constexpr uint64_t kSegPerLaunch = (uint64_t)tnc::kSegHeader + tnc::kMaxArgBytes;

struct RingLayout {
  uint64_t per_ws = 0, per_out = 0, seg = 0, total = 0;
  int group = 1;
};

// Workspace of one call: [segment tables | G slice workspaces | G slice
// results]; `launches` is one slice's launch count.
int ring_layout(tnc_ring_plan_t ring, int32_t k, int32_t n_batches, uint64_t launches, RingLayout* L) {
  uint64_t ws = 0;
  const int rc = tnc_workspace_bytes(ring->slices[0], k, n_batches, TNC_STORE_C64, &ws);
  if (rc) return rc;
  L->per_ws = align256(ws);
  L->per_out = align256((uint64_t)n_batches << k << 4);
  const uint64_t per = L->per_ws + L->per_out + launches * kSegPerLaunch;
  L->group = (int)std::max<uint64_t>(1, std::min<uint64_t>({(uint64_t)ring->slices.size(), (uint64_t)kMaxGroup,
                                                            kGroupBytes / per}));
  L->seg = align256((uint64_t)L->group * launches * kSegPerLaunch);
  L->total = L->seg + (uint64_t)L->group * (L->per_ws + L->per_out);
  return TNC_OK;
}

// At most the launches of one slice's amplitude call with its whole
// workspace (build-up, variant resolution, passes, late launches; the same
// for every slice), from the plan alone (no device involved).
int slice_launches(tnc_ring_plan_t ring, int32_t k, int32_t n_batches, uint64_t* count) {
  (void)n_batches;
  tnc_info info;
  const int rc = tnc_plan_info(ring->slices[0], k, &info);
  if (rc) return rc;
  *count = 2 + (uint64_t)info.n_passes + (uint64_t)info.n_late_launches;
  return TNC_OK;
}

// out = L * X for 2x2 row-major complex matrices.
void right_mul(tnc_c128* L, const std::complex<double> X[4]) {
  std::complex<double> a[4], r[4];
  for (int e = 0; e < 4; ++e) a[e] = {L[e].re, L[e].im};
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j) r[2 * i + j] = a[2 * i] * X[j] + a[2 * i + 1] * X[2 + j];
  for (int e = 0; e < 4; ++e) L[e] = tnc_c128{r[e].real(), r[e].imag()};
}

}  // namespace

extern "C" {

int tnc_plan_ring(int32_t n, int32_t d, const tnc_c128* one_qubit, int32_t n_gate2, const tnc_gate2* gates,
                  const tnc_options* opt, tnc_ring_plan_t* out) {
  if (!out || !one_qubit || (n_gate2 > 0 && !gates)) return ring_err(TNC_E_INVALID, "null argument");
  *out = nullptr;
  if (n < 3 || d < 1) return ring_err(TNC_E_DOMAIN, "a ring needs n >= 3 and d >= 1");
  std::vector<tnc_gate2> chain;
  std::vector<int> cut_layers;
  for (int i = 0; i < n_gate2; ++i) {
    if (gates[i].q == n - 1) {
      if (gates[i].kind != TNC_GATE_CZ) return ring_err(TNC_E_INVALID, "wrap-pair gates must be CZ");
      if (gates[i].layer < 1 || gates[i].layer > d) return ring_err(TNC_E_INVALID, "wrap gate layer out of range");
      for (int l : cut_layers)
        if (l == gates[i].layer) return ring_err(TNC_E_INVALID, "two wrap gates in one layer");
      cut_layers.push_back(gates[i].layer);
    } else {
      chain.push_back(gates[i]);
    }
  }
  const int m = (int)cut_layers.size();
  if (m > 12) return ring_err(TNC_E_DOMAIN, "more than 12 wrap gates (2^12 slices)");
  // qubits n-1 and 0 must be idle in the chain pattern of every cut layer
  for (const tnc_gate2& g : chain)
    for (int l : cut_layers)
      if (g.layer == l && (g.q == 0 || g.q + 1 == n - 1))
        return ring_err(TNC_E_INVALID, "a wrap gate's qubits must be idle in the chain pattern of its layer");
  auto* rp = new tnc_ring_plan_s();
  rp->n = n;
  rp->d = d;
  rp->m = m;
  const size_t one_n = (size_t)(d + 1) * n * 4;
  std::vector<tnc_c128> one(one_n);
  for (int a = 0; a < (1 << m); ++a) {
    std::memcpy(one.data(), one_qubit, one_n * sizeof(tnc_c128));
    for (int j = 0; j < m; ++j) {
      const int bit = (a >> j) & 1;
      const int l = cut_layers[j];
      const std::complex<double> P[4] = {double(1 - bit), 0.0, 0.0, double(bit)};  // |a><a| on q_{n-1}
      const std::complex<double> Z[4] = {1.0, 0.0, 0.0, bit ? -1.0 : 1.0};          // Z^a on q_0
      right_mul(one.data() + ((size_t)l * n + (n - 1)) * 4, P);
      right_mul(one.data() + ((size_t)l * n + 0) * 4, Z);
    }
    tnc_plan_t p = nullptr;
    const int rc = tnc_plan(n, d, one.data(), (int32_t)chain.size(), chain.data(), opt, &p);
    if (rc) {
      tnc_ring_release(rp);
      return rc;
    }
    rp->slices.push_back(p);
  }
  *out = rp;
  return TNC_OK;
}

int tnc_ring_info(tnc_ring_plan_t ring, int32_t k, int32_t n_batches, int32_t* n_slices, int32_t* width,
                  uint64_t* workspace_bytes) {
  if (!ring || ring->slices.empty()) return ring_err(TNC_E_INVALID, "null ring plan");
  if (n_batches < 1) return ring_err(TNC_E_INVALID, "n_batches < 1");
  tnc_info info;
  int rc = tnc_plan_info(ring->slices[0], k, &info);
  if (rc) return rc;
  uint64_t launches = 0;
  if ((rc = slice_launches(ring, k, n_batches, &launches))) return rc;
  RingLayout L;
  if ((rc = ring_layout(ring, k, n_batches, launches, &L))) return rc;
  if (n_slices) *n_slices = (int32_t)ring->slices.size();
  if (width) *width = info.width;
  if (workspace_bytes) *workspace_bytes = L.total;
  return TNC_OK;
}

int tnc_ring_amplitudes(tnc_ring_plan_t ring, int32_t n_batches, const uint8_t* d_bits, int32_t k, tnc_c128* d_out,
                        void* d_workspace, uint64_t workspace_bytes, void* stream) {
  if (!ring || ring->slices.empty()) return ring_err(TNC_E_INVALID, "null ring plan");
  if (n_batches < 0) return ring_err(TNC_E_INVALID, "n_batches < 0");
  if (n_batches == 0) return TNC_OK;
  if (!d_bits || !d_out || !d_workspace) return ring_err(TNC_E_INVALID, "null argument");
  uint64_t launches = 0;
  int rc = slice_launches(ring, k, n_batches, &launches);
  if (rc) return rc;
  RingLayout L;
  if ((rc = ring_layout(ring, k, n_batches, launches, &L))) return rc;
  if (workspace_bytes < L.total) return ring_err(TNC_E_NOMEM, "ring workspace smaller than tnc_ring_info reports");
  uint64_t ws = 0;
  if ((rc = tnc_workspace_bytes(ring->slices[0], k, n_batches, TNC_STORE_C64, &ws))) return rc;
  char* base = static_cast<char*>(d_workspace);
  char* ws_base = base + L.seg;
  char* out_base = ws_base + (uint64_t)L.group * L.per_ws;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const long long count = (long long)n_batches << k;
  hipError_t e = tnc::launch_fill_zero(reinterpret_cast<double2*>(d_out), count, s);
  if (e != hipSuccess) return ring_err(TNC_E_DEVICE, hipGetErrorString(e));
  if (ring->h_cap < L.seg) {
    if (ring->copied) (void)hipEventSynchronize(ring->copied);
    if (ring->h_seg) (void)hipHostFree(ring->h_seg);
    ring->h_seg = nullptr;
    ring->h_cap = 0;
    if ((e = hipHostMalloc((void**)&ring->h_seg, L.seg)) != hipSuccess) return ring_err(TNC_E_NOMEM, "pinned staging");
    ring->h_cap = L.seg;
  }
  if (!ring->copied && (e = hipEventCreateWithFlags(&ring->copied, hipEventDisableTiming)) != hipSuccess)
    return ring_err(TNC_E_DEVICE, hipGetErrorString(e));
  const int n_sl = (int)ring->slices.size();
  for (int g0 = 0; g0 < n_sl; g0 += L.group) {
    const int G = std::min(L.group, n_sl - g0);
    // every slice of the group recorded against its own workspace and result
    std::vector<std::vector<tnc::Launch>> ls(G);
    for (int i = 0; i < G; ++i) {
      rc = tnc::record_amplitudes(ring->slices[g0 + i], n_batches, d_bits, k, TNC_STORE_C64,
                                  reinterpret_cast<tnc_c128*>(out_base + (uint64_t)i * L.per_out),
                                  ws_base + (uint64_t)i * L.per_ws, ws, &ls[i]);
      if (rc) return rc;
      if (ls[i].size() != ls[0].size() || ls[i].size() > launches)
        return ring_err(TNC_E_INVALID, "ring slices of different shapes");
    }
    // the previous group's table upload has finished before its staging is rewritten
    if ((e = hipEventSynchronize(ring->copied)) != hipSuccess) return ring_err(TNC_E_DEVICE, hipGetErrorString(e));
    std::vector<std::vector<const tnc::Launch*>> steps(ls[0].size());
    std::vector<uint64_t> seg_off(ls[0].size(), 0);
    uint64_t seg_at = 0;
    for (size_t j = 0; j < ls[0].size(); ++j) {
      for (int i = 0; i < G; ++i) {
        if (!tnc::groupable(ls[0][j], ls[i][j])) return ring_err(TNC_E_INVALID, "ring slices of different launches");
        steps[j].push_back(&ls[i][j]);
      }
      if (G < 2) continue;
      const uint64_t need = (uint64_t)G * ls[0][j].seg_stride;
      if (seg_at + need > L.seg) return ring_err(TNC_E_NOMEM, "ring segment tables");
      seg_off[j] = seg_at;
      tnc::write_segments(steps[j].data(), G, ring->h_seg + seg_at);
      seg_at = align256(seg_at + need);
    }
    if (seg_at > 0) {
      if ((e = hipMemcpyAsync(base, ring->h_seg, seg_at, hipMemcpyHostToDevice, s)) != hipSuccess)
        return ring_err(TNC_E_DEVICE, hipGetErrorString(e));
    }
    if ((e = hipEventRecord(ring->copied, s)) != hipSuccess) return ring_err(TNC_E_DEVICE, hipGetErrorString(e));
    for (size_t j = 0; j < steps.size(); ++j) {
      if (G < 2) {
        std::vector<tnc::Launch> one(1, *steps[j][0]);
        if ((rc = tnc::issue_recorded(one, s))) return rc;
        continue;
      }
      if ((e = tnc::issue_grouped(steps[j].data(), G, base + seg_off[j], s)) != hipSuccess)
        return ring_err(TNC_E_DEVICE, hipGetErrorString(e));
    }
    // the group's results added to the sum, slice by slice in index order
    e = tnc::launch_accumulate_rows(reinterpret_cast<double2*>(d_out), reinterpret_cast<const double2*>(out_base),
                                    L.per_out / sizeof(double2), G, count, s);
    if (e != hipSuccess) return ring_err(TNC_E_DEVICE, hipGetErrorString(e));
  }
  return TNC_OK;
}

int tnc_debug_ring_emulate(tnc_ring_plan_t ring, int32_t n_batches, const uint8_t* bits, int32_t k,
                           tnc_c128* out) {
  if (!ring || ring->slices.empty()) return ring_err(TNC_E_INVALID, "null ring plan");
  if (n_batches < 0 || (n_batches > 0 && (!bits || !out))) return ring_err(TNC_E_INVALID, "bad argument");
  const size_t count = (size_t)n_batches << k;
  std::vector<tnc_c128> part(count);
  for (size_t i = 0; i < count; ++i) out[i] = tnc_c128{0.0, 0.0};
  for (tnc_plan_t p : ring->slices) {
    const int rc = tnc_debug_emulate_device(p, n_batches, bits, k, TNC_STORE_C64, part.data());
    if (rc) return rc;
    for (size_t i = 0; i < count; ++i) {
      out[i].re += part[i].re;
      out[i].im += part[i].im;
    }
  }
  return TNC_OK;
}

void tnc_ring_release(tnc_ring_plan_t ring) {
  if (!ring) return;
  if (ring->copied) {
    (void)hipEventSynchronize(ring->copied);
    (void)hipEventDestroy(ring->copied);
  }
  if (ring->h_seg) (void)hipHostFree(ring->h_seg);
  for (tnc_plan_t p : ring->slices) tnc_release(p);
  delete ring;
}

}  // extern "C"
