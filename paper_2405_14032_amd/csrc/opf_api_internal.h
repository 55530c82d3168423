// Model accessors shared by the ABI translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/opf.h"
#include "opf_host.h"

namespace opf {
// Records msg as the thread's last error and returns code.
int api_fail(int code, const std::string& msg);
int model_device(const opf_model* M);  // < 0: host-only model
hipStream_t model_stream(const opf_model* M);
const std::vector<InstHost>& model_insts(const opf_model* M);
int64_t model_n(const opf_model* M);
int64_t model_nnzk(const opf_model* M);
const opf_model* chol_model(const opf_chol* F);  // the model F was analysed from
}  // namespace opf
