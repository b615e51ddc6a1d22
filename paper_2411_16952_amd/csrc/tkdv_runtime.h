// Runtime services of the context shared by the library's source files.
#pragma once

#include <string>

#include "../../include/tkdv.h"

namespace tkdv {

int ctx_device(const tkdv_ctx *ctx);
// Records msg as the text of the last context-less error and returns st.
tkdv_status record_error(tkdv_status st, const std::string &msg);

}  // namespace tkdv
