// Ring geometry by structure-aware slicing (Sec. 6.3): the CZ gates of the
// wrap pair (n-1, 0) are cut, CZ = sum_a P_a (x) Z^a with P_a = |a><a| on
// qubit n-1 and Z^a on qubit 0.  Each of the 2^m assignments of the m cut
// bonds is an open-chain circuit (its P_a, Z^a factors folded into the
// one-qubit layer that follows the cut gate, where both qubits are idle in
// the chain pattern), planned and contracted like any other; the ring's
// amplitudes are the sum over the slices.  Built on the public C ABI.
#include <hip/hip_runtime.h>

#include <complex>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/tnc.h"
#include "kernels.hpp"

namespace tnc {
int set_error_message(int code, const std::string& msg);
}

struct tnc_ring_plan_s {
  int n = 0, d = 0, m = 0;
  std::vector<tnc_plan_t> slices;
};

namespace {

int ring_err(int code, const char* msg) { return tnc::set_error_message(code, msg); }

uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

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
  tnc_info info;
  int rc = tnc_plan_info(ring->slices[0], k, &info);
  if (rc) return rc;
  uint64_t ws = 0;
  if ((rc = tnc_workspace_bytes(ring->slices[0], k, n_batches, TNC_STORE_C64, &ws))) return rc;
  if (n_slices) *n_slices = (int32_t)ring->slices.size();
  if (width) *width = info.width;
  if (workspace_bytes) *workspace_bytes = align256(ws) + align256((uint64_t)n_batches << k << 4);
  return TNC_OK;
}

int tnc_ring_amplitudes(tnc_ring_plan_t ring, int32_t n_batches, const uint8_t* d_bits, int32_t k, tnc_c128* d_out,
                        void* d_workspace, uint64_t workspace_bytes, void* stream) {
  if (!ring || ring->slices.empty()) return ring_err(TNC_E_INVALID, "null ring plan");
  if (n_batches < 0) return ring_err(TNC_E_INVALID, "n_batches < 0");
  if (n_batches == 0) return TNC_OK;
  if (!d_bits || !d_out || !d_workspace) return ring_err(TNC_E_INVALID, "null argument");
  uint64_t ws = 0;
  int rc = tnc_workspace_bytes(ring->slices[0], k, n_batches, TNC_STORE_C64, &ws);
  if (rc) return rc;
  const uint64_t tmp_bytes = (uint64_t)n_batches << k << 4;
  if (workspace_bytes < align256(ws) + align256(tmp_bytes))
    return ring_err(TNC_E_NOMEM, "ring workspace smaller than tnc_ring_info reports");
  char* base = static_cast<char*>(d_workspace);
  auto* tmp = reinterpret_cast<tnc_c128*>(base + align256(ws));
  hipStream_t s = static_cast<hipStream_t>(stream);
  const long long count = (long long)n_batches << k;
  hipError_t e = tnc::launch_fill_zero(reinterpret_cast<double2*>(d_out), count, s);
  if (e != hipSuccess) return ring_err(TNC_E_DEVICE, hipGetErrorString(e));
  // slices in index order, each added to the sum once its batch is out
  for (tnc_plan_t p : ring->slices) {
    if ((rc = tnc_amplitudes(p, n_batches, d_bits, k, TNC_STORE_C64, tmp, base, ws, stream))) return rc;
    e = tnc::launch_accumulate(reinterpret_cast<double2*>(d_out), reinterpret_cast<const double2*>(tmp), count, s);
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
  for (tnc_plan_t p : ring->slices) tnc_release(p);
  delete ring;
}

}  // extern "C"
