// Declarations shared by the library's own sources (not part of the C ABI).
#pragma once

#include <cstdint>

#include "iqa.h"

namespace iqa {

// iqa_batch_describe with the per-pair geometry of tuned kind `kind`
// (IQA_TUNE_BATCH: the ragged-batch geometry; IQA_TUNE_SERVE: the server's).
iqa_status describe_pairs(const iqa_pair *pairs, int64_t count, void *descs,
                          int64_t *total_units, int kind);

}  // namespace iqa
