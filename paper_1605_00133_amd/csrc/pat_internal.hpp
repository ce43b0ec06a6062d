// Internal host-side declarations shared by the C-ABI translation units.
#pragma once

#include <cstdint>

#include "../../include/pat.h"

namespace pat {

// Records a message for pat_last_error() and returns `st`.
pat_status set_error(pat_status st, const char* fmt, ...);

pat_status make_rsp_mask(int32_t n_pix, int32_t mc, uint64_t seed, int32_t* idx_out);
pat_status make_shd_pattern(int32_t n_pix, int32_t mc, uint64_t seed, int32_t* perm_out, int32_t* rows_out);

}  // namespace pat
