// Stencil instantiations: FP64 spinors with 18- or 12-real FP64 links (and the 12-real links read non-temporally), adjoint hopping.
#include "dslash_impl.h"

namespace wd {

hipError_t dslash_launch_f64_d1(const DslashArgs &a, int lk, int nr, int rl, int epi, int block,
                              int grid, hipStream_t s)
{
    if (lk == LK_F64_18) {
        WD_DSL_SHAPE(SP_F64, LK_F64_18, 1, 1, true)
        WD_DSL_SHAPE(SP_F64, LK_F64_18, 2, 1, true)
        WD_DSL_SHAPE(SP_F64, LK_F64_18, 1, 2, true)
        WD_DSL_SHAPE(SP_F64, LK_F64_18, 2, 2, true)
        WD_DSL_SHAPE(SP_F64, LK_F64_18, 1, 4, true)
        WD_DSL_SHAPE(SP_F64, LK_F64_18, 2, 4, true)
    }
    if (lk == LK_F64_12) {
        WD_DSL_SHAPE(SP_F64, LK_F64_12, 1, 1, true)
        WD_DSL_SHAPE(SP_F64, LK_F64_12, 2, 1, true)
        WD_DSL_SHAPE(SP_F64, LK_F64_12, 1, 2, true)
        WD_DSL_SHAPE(SP_F64, LK_F64_12, 2, 2, true)
        WD_DSL_SHAPE(SP_F64, LK_F64_12, 1, 4, true)
        WD_DSL_SHAPE(SP_F64, LK_F64_12, 2, 4, true)
    }
    if (lk == LK_F64_12N) {
        WD_DSL_SHAPE(SP_F64, LK_F64_12N, 1, 1, true)
        WD_DSL_SHAPE(SP_F64, LK_F64_12N, 2, 1, true)
    }
    return hipErrorInvalidValue;
}

}  // namespace wd
