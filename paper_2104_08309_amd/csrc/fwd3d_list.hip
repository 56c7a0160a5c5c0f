// The FP32C single-mesh forward in the list order of the faces (no edge sharing): the instance of
// fwd3d_fp32c_kernel that this file compiles with the instruction-level-parallelism scheduler, under
// which it runs faster than under the default one (the edge-sharing instance in fwd3d.hip the other
// way round).
#include "fwd3d_fp32c.h"

namespace pft {

hipError_t launch_fwd3d_fp32c_list(const FwdArgs& a, hipStream_t s) {
  const int64_t qtiles = (a.nq + kFwdQTile - 1) / kFwdQTile;
  const int64_t blocks = (qtiles + kXcds - 1) / kXcds * kXcds * a.splits;
  if (blocks > 0x7fffffff) return hipErrorInvalidConfiguration;
  fwd3d_fp32c_kernel<false><<<(unsigned)blocks, kFwdBlock, 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace pft
