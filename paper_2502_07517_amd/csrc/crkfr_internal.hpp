// Declarations shared by the host translation units of libcrkfr (not part of
// the C ABI).
#pragma once
#include <string>

#include "../../include/crkfr.h"

namespace crkfr {

// record the message returned by crkfr_last_error and pass the code through
int set_error(int code, const std::string& msg);

// the learned indicator's network as the step kernels read it: device
// parameters followed by the feature box lo[n_inputs], hi[n_inputs]
const float* mlp_device_params(const crkfr_mlp* m);
int mlp_inputs(const crkfr_mlp* m);
int mlp_hidden(const crkfr_mlp* m);

}  // namespace crkfr
