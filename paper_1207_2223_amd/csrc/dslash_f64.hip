// FP64 instantiations of the hopping stencil: 18- or 12-real FP64 links.
#include "dslash_impl.h"

namespace wd {

hipError_t dslash_launch_f64(const DslashArgs &a, int lk, int nr, int dag, int epi, int block,
                             int grid, hipStream_t s)
{
    if (lk == LK_F64_18) {
        if (nr == 1) { WD_DSL_DAG(SP_F64, LK_F64_18, 1, SP_F64) }
        if (nr == 2) { WD_DSL_DAG(SP_F64, LK_F64_18, 2, SP_F64) }
    } else if (lk == LK_F64_12) {
        if (nr == 1) { WD_DSL_DAG(SP_F64, LK_F64_12, 1, SP_F64) }
        if (nr == 2) { WD_DSL_DAG(SP_F64, LK_F64_12, 2, SP_F64) }
    }
    return hipErrorInvalidValue;
}

}  // namespace wd
