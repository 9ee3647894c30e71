// gsf_merged_bf16.hip -- merged spatial sweeps with bfloat16 F storage (instantiations
// of gsf_merged.h, one file per storage type so they compile in parallel).
#include "gsf_merged.h"

namespace gsf {

MergedFn merged_fn_bf16(int form, int shape) { return merged::lookup<__bf16>(form, shape); }

}  // namespace gsf
