// gsf_merged_f16.hip -- merged spatial sweeps with binary16 F storage (instantiations
// of gsf_merged.h, one file per storage type so they compile in parallel).
#include "gsf_merged.h"

namespace gsf {

MergedFn merged_fn_f16(int form, int shape) { return merged::lookup<_Float16>(form, shape); }

}  // namespace gsf
