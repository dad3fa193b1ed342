// Stencil instantiations: FP16 spinors (per-site FP32 norm) with FP32 12-real, FP32 18-real, FP16 12-real or FP32 8-real links (and FP32 12- and 8-real links read non-temporally), forward hopping.
#include "dslash_impl.h"

namespace wd {

hipError_t dslash_launch_f16_d0(const DslashArgs &a, int lk, int nr, int rl, int epi, int block,
                              int grid, hipStream_t s)
{
    if (lk == LK_F32_12) {
        WD_DSL_SHAPE(SP_F16, LK_F32_12, 1, 1, false)
        WD_DSL_SHAPE(SP_F16, LK_F32_12, 2, 1, false)
        WD_DSL_SHAPE(SP_F16, LK_F32_12, 3, 1, false)
        WD_DSL_SHAPE(SP_F16, LK_F32_12, 4, 1, false)
        WD_DSL_SHAPE(SP_F16, LK_F32_12, 1, 2, false)
        WD_DSL_SHAPE(SP_F16, LK_F32_12, 2, 2, false)
        WD_DSL_SHAPE(SP_F16, LK_F32_12, 3, 2, false)
        WD_DSL_SHAPE(SP_F16, LK_F32_12, 4, 2, false)
        WD_DSL_SHAPE(SP_F16, LK_F32_12, 1, 4, false)
        WD_DSL_SHAPE(SP_F16, LK_F32_12, 2, 4, false)
        WD_DSL_SHAPE(SP_F16, LK_F32_12, 3, 4, false)
        WD_DSL_SHAPE(SP_F16, LK_F32_12, 4, 4, false)
    }
    if (lk == LK_F16_12) {
        WD_DSL_SHAPE(SP_F16, LK_F16_12, 1, 1, false)
        WD_DSL_SHAPE(SP_F16, LK_F16_12, 2, 1, false)
        WD_DSL_SHAPE(SP_F16, LK_F16_12, 3, 1, false)
        WD_DSL_SHAPE(SP_F16, LK_F16_12, 4, 1, false)
        WD_DSL_SHAPE(SP_F16, LK_F16_12, 1, 2, false)
        WD_DSL_SHAPE(SP_F16, LK_F16_12, 2, 2, false)
        WD_DSL_SHAPE(SP_F16, LK_F16_12, 3, 2, false)
        WD_DSL_SHAPE(SP_F16, LK_F16_12, 4, 2, false)
        WD_DSL_SHAPE(SP_F16, LK_F16_12, 1, 4, false)
        WD_DSL_SHAPE(SP_F16, LK_F16_12, 2, 4, false)
        WD_DSL_SHAPE(SP_F16, LK_F16_12, 3, 4, false)
        WD_DSL_SHAPE(SP_F16, LK_F16_12, 4, 4, false)
    }
    if (lk == LK_F32_18) {
        WD_DSL_SHAPE(SP_F16, LK_F32_18, 1, 1, false)
        WD_DSL_SHAPE(SP_F16, LK_F32_18, 2, 1, false)
        WD_DSL_SHAPE(SP_F16, LK_F32_18, 3, 1, false)
        WD_DSL_SHAPE(SP_F16, LK_F32_18, 4, 1, false)
        WD_DSL_SHAPE(SP_F16, LK_F32_18, 1, 2, false)
        WD_DSL_SHAPE(SP_F16, LK_F32_18, 2, 2, false)
        WD_DSL_SHAPE(SP_F16, LK_F32_18, 3, 2, false)
        WD_DSL_SHAPE(SP_F16, LK_F32_18, 4, 2, false)
        WD_DSL_SHAPE(SP_F16, LK_F32_18, 1, 4, false)
        WD_DSL_SHAPE(SP_F16, LK_F32_18, 2, 4, false)
        WD_DSL_SHAPE(SP_F16, LK_F32_18, 3, 4, false)
        WD_DSL_SHAPE(SP_F16, LK_F32_18, 4, 4, false)
    }
    if (lk == LK_F32_8) {
        WD_DSL_SHAPE(SP_F16, LK_F32_8, 1, 1, false)
        WD_DSL_SHAPE(SP_F16, LK_F32_8, 2, 1, false)
        WD_DSL_SHAPE(SP_F16, LK_F32_8, 1, 2, false)
        WD_DSL_SHAPE(SP_F16, LK_F32_8, 2, 2, false)
        WD_DSL_SHAPE(SP_F16, LK_F32_8, 1, 4, false)
        WD_DSL_SHAPE(SP_F16, LK_F32_8, 2, 4, false)
    }
    if (lk == LK_F32_12N) {
        WD_DSL_SHAPE(SP_F16, LK_F32_12N, 1, 1, false)
        WD_DSL_SHAPE(SP_F16, LK_F32_12N, 2, 1, false)
    }
    if (lk == LK_F32_8N) {
        WD_DSL_SHAPE(SP_F16, LK_F32_8N, 1, 1, false)
        WD_DSL_SHAPE(SP_F16, LK_F32_8N, 2, 1, false)
    }
    return hipErrorInvalidValue;
}

// The LDS-staged t-walking instances (RL = 1).
hipError_t dslash_lds_launch_f16_d0(const DslashArgs &a, int lk, int nr, int epi, int grid, unsigned lds_bytes,
                                  hipStream_t s)
{
    if (lk == LK_F32_12) {
        WD_DSL_LDS_SHAPE(SP_F16, LK_F32_12, 1, false)
        WD_DSL_LDS_SHAPE(SP_F16, LK_F32_12, 2, false)
    }
    if (lk == LK_F16_12) {
        WD_DSL_LDS_SHAPE(SP_F16, LK_F16_12, 1, false)
        WD_DSL_LDS_SHAPE(SP_F16, LK_F16_12, 2, false)
    }
    return hipErrorInvalidValue;
}

}  // namespace wd
