// gsf_merged_f32.hip -- merged spatial sweeps with FP32 F storage (instantiations
// of gsf_merged.h, one file per storage type so they compile in parallel).
#include "gsf_merged.h"

namespace gsf {

MergedFn merged_fn_f32(int form, int shape) { return merged::lookup<float>(form, shape); }

}  // namespace gsf
