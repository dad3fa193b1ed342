// Stencil instantiations: FP64 spinors with 18- or 12-real FP64 links (and the 12-real links read non-temporally), forward hopping.
#include "dslash_impl.h"

namespace wd {

hipError_t dslash_launch_f64_d0(const DslashArgs &a, int lk, int nr, int rl, int epi, int block,
                              int grid, hipStream_t s)
{
    if (lk == LK_F64_18) {
        WD_DSL_SHAPE(SP_F64, LK_F64_18, 1, 1, false)
        WD_DSL_SHAPE(SP_F64, LK_F64_18, 2, 1, false)
        WD_DSL_SHAPE(SP_F64, LK_F64_18, 1, 2, false)
        WD_DSL_SHAPE(SP_F64, LK_F64_18, 2, 2, false)
        WD_DSL_SHAPE(SP_F64, LK_F64_18, 1, 4, false)
        WD_DSL_SHAPE(SP_F64, LK_F64_18, 2, 4, false)
    }
    if (lk == LK_F64_12) {
        WD_DSL_SHAPE(SP_F64, LK_F64_12, 1, 1, false)
        WD_DSL_SHAPE(SP_F64, LK_F64_12, 2, 1, false)
        WD_DSL_SHAPE(SP_F64, LK_F64_12, 1, 2, false)
        WD_DSL_SHAPE(SP_F64, LK_F64_12, 2, 2, false)
        WD_DSL_SHAPE(SP_F64, LK_F64_12, 1, 4, false)
        WD_DSL_SHAPE(SP_F64, LK_F64_12, 2, 4, false)
    }
    if (lk == LK_F64_12N) {
        WD_DSL_SHAPE(SP_F64, LK_F64_12N, 1, 1, false)
        WD_DSL_SHAPE(SP_F64, LK_F64_12N, 2, 1, false)
    }
    return hipErrorInvalidValue;
}

}  // namespace wd
