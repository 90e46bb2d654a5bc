// Reduced-precision form (fp16 / bf16 MFMA transforms with an int8 residual plane).
#include "sf_internal.h"

namespace sf {

int launch_frag_lp(const DeviceState &, const Geom &, const uint8_t *, void *, uint8_t *, int8_t *, const AesArgs &,
                   uint32_t *, hipStream_t) {
  return fail(SF_ENOTSUP, "reduced-precision form not built yet");
}

int launch_defrag_lp(const DeviceState &, const Geom &, const void *, const uint8_t *, const int8_t *,
                     const AesArgs &, uint8_t *, uint32_t *, hipStream_t) {
  return fail(SF_ENOTSUP, "reduced-precision form not built yet");
}

}  // namespace sf
