// Tile autotuner: times candidate pass tilings on the device.
//
// The width, the op sequence and hence the pass partition depend only on the
// circuit's shape (n, d) and k, not on its gate values: one-qubit gates,
// T gates included, are absorbed without changing the network (Sec. 1 and
// Sec. 7).  So one synthetic circuit of the right shape stands for every
// circuit of that shape: brickwork CZ layers with seeded random one-qubit
// unitaries.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <limits>
#include <vector>

#include "tnc.h"

namespace {

// SplitMix64 (Steele, Lea, Flood 2014).
struct SplitMix64 {
  uint64_t s;
  uint64_t next() {
    uint64_t z = (s += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
  }
  double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

// A unitary 2x2 from three angles: [[c, -e^{il} s], [e^{ip} s, e^{i(p+l)} c]].
void random_u2(SplitMix64& g, tnc_c128* m) {
  const double th = std::acos(std::sqrt(g.uniform())), ph = 2 * M_PI * g.uniform(), la = 2 * M_PI * g.uniform();
  const double c = std::cos(th), s = std::sin(th);
  m[0] = {c, 0.0};
  m[1] = {-std::cos(la) * s, -std::sin(la) * s};
  m[2] = {std::cos(ph) * s, std::sin(ph) * s};
  m[3] = {std::cos(ph + la) * c, std::sin(ph + la) * c};
}

}  // namespace

extern "C" int tnc_autotune(int32_t n, int32_t d, int32_t k, int32_t storage, const tnc_options* candidates,
                            int32_t n_candidates, int32_t reps, int32_t* best, double* times_ms) {
  if (n < 2 || d < 2 || !candidates || n_candidates < 1 || reps < 1 || !best || !times_ms) return TNC_E_INVALID;
  SplitMix64 g{0x7A3C5ull ^ ((uint64_t)n << 20) ^ (uint64_t)d};
  std::vector<tnc_c128> one((size_t)(d + 1) * n * 4);
  for (size_t q = 0; q < one.size(); q += 4) random_u2(g, one.data() + q);
  std::vector<tnc_gate2> gates;
  for (int l = 1; l <= d; ++l)
    for (int q = (l & 1) ? 1 : 0; q + 1 < n; q += 2) {
      tnc_gate2 t{};
      t.layer = l;
      t.q = q;
      t.kind = TNC_GATE_CZ;
      gates.push_back(t);
    }
  std::vector<uint8_t> bits((size_t)n, 0);
  uint8_t* d_bits = nullptr;
  tnc_c128* d_out = nullptr;
  if (hipMalloc((void**)&d_bits, bits.size()) != hipSuccess) return TNC_E_NOMEM;
  if (hipMalloc((void**)&d_out, sizeof(tnc_c128) << k) != hipSuccess) {
    (void)hipFree(d_bits);
    return TNC_E_NOMEM;
  }
  (void)hipMemcpy(d_bits, bits.data(), bits.size(), hipMemcpyHostToDevice);
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  int rc = TNC_OK;
  if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess || hipEventCreate(&e0) != hipSuccess ||
      hipEventCreate(&e1) != hipSuccess)
    rc = TNC_E_DEVICE;
  int32_t bi = -1;
  for (int c = 0; c < n_candidates && rc == TNC_OK; ++c) {
    times_ms[c] = std::numeric_limits<double>::infinity();
    tnc_plan_t p = nullptr;
    if (tnc_plan(n, d, one.data(), (int32_t)gates.size(), gates.data(), &candidates[c], &p) != TNC_OK) continue;
    uint64_t ws = 0;
    void* d_ws = nullptr;
    if (tnc_prepare(p, k) == TNC_OK && tnc_workspace_bytes(p, k, 1, storage, &ws) == TNC_OK &&
        hipMalloc(&d_ws, ws) == hipSuccess) {
      std::vector<double> t;
      bool ok = tnc_amplitudes(p, 1, d_bits, k, storage, d_out, d_ws, ws, st) == TNC_OK &&
                hipStreamSynchronize(st) == hipSuccess;
      for (int r = 0; r < reps && ok; ++r) {
        float ms = 0.f;
        ok = hipEventRecord(e0, st) == hipSuccess &&
             tnc_amplitudes(p, 1, d_bits, k, storage, d_out, d_ws, ws, st) == TNC_OK &&
             hipEventRecord(e1, st) == hipSuccess && hipEventSynchronize(e1) == hipSuccess &&
             hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
        if (ok) t.push_back(ms);
      }
      if (ok && !t.empty()) {
        std::sort(t.begin(), t.end());
        times_ms[c] = t[t.size() / 2];
        if (bi < 0 || times_ms[c] < times_ms[bi]) bi = c;
      }
    }
    if (d_ws) (void)hipFree(d_ws);
    tnc_release(p);
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st) (void)hipStreamDestroy(st);
  (void)hipFree(d_bits);
  (void)hipFree(d_out);
  if (rc != TNC_OK) return rc;
  if (bi < 0) return TNC_E_INVALID;
  *best = bi;
  return TNC_OK;
}
