// Internal interface between the C ABI (tnc_api.cpp) and the serving loop
// (serve.cpp): the launches of an amplitude call as records.
#pragma once

#include <string>
#include <vector>

#include "../../include/tnc.h"
#include "kernels.hpp"

namespace tnc {

// Records every launch that tnc_amplitudes would issue for these arguments,
// in order, without issuing any (the device tables for k are built and
// uploaded on first use).  Returns TNC_OK or the status tnc_amplitudes
// would return.
int record_amplitudes(tnc_plan_t plan, int32_t n_batches, const uint8_t* d_bits, int32_t k, int32_t storage,
                      tnc_c128* d_out, void* d_workspace, uint64_t workspace_bytes, std::vector<Launch>* out);

// Issues recorded launches in order on `stream` (timed while profiling is
// on); TNC_E_DEVICE with the failing launch's own status.
int issue_recorded(const std::vector<Launch>& ls, hipStream_t stream);

// Sets the calling thread's error message (tnc_last_error) and returns code.
int set_error_message(int code, const std::string& msg);

}  // namespace tnc
