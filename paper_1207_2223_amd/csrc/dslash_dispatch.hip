// Stencil launch dispatch over spinor precision and dagger.
#include "wd_internal.h"

namespace wd {

hipError_t dslash_launch_f64_d0(const DslashArgs &a, int lk, int nr, int rl, int epi, int block, int grid, hipStream_t s);
hipError_t dslash_launch_f64_d1(const DslashArgs &a, int lk, int nr, int rl, int epi, int block, int grid, hipStream_t s);
hipError_t dslash_launch_f32_d0(const DslashArgs &a, int lk, int nr, int rl, int epi, int block, int grid, hipStream_t s);
hipError_t dslash_launch_f32_d1(const DslashArgs &a, int lk, int nr, int rl, int epi, int block, int grid, hipStream_t s);
hipError_t dslash_launch_f16_d0(const DslashArgs &a, int lk, int nr, int rl, int epi, int block, int grid, hipStream_t s);
hipError_t dslash_launch_f16_d1(const DslashArgs &a, int lk, int nr, int rl, int epi, int block, int grid, hipStream_t s);
hipError_t dslash_launch_i16_d0(const DslashArgs &a, int lk, int nr, int rl, int epi, int block, int grid, hipStream_t s);
hipError_t dslash_launch_i16_d1(const DslashArgs &a, int lk, int nr, int rl, int epi, int block, int grid, hipStream_t s);

hipError_t dslash_lds_launch_f16_d0(const DslashArgs &a, int lk, int nr, int epi, int grid, unsigned lds_bytes, hipStream_t s);
hipError_t dslash_lds_launch_f16_d1(const DslashArgs &a, int lk, int nr, int epi, int grid, unsigned lds_bytes, hipStream_t s);
hipError_t dslash_lds_launch_f32_d0(const DslashArgs &a, int lk, int nr, int epi, int grid, unsigned lds_bytes, hipStream_t s);
hipError_t dslash_lds_launch_f32_d1(const DslashArgs &a, int lk, int nr, int epi, int grid, unsigned lds_bytes, hipStream_t s);

hipError_t dslash_tw_launch_f16_d0(const DslashArgs &a, int lk, int nr, int epi, int block, int grid, hipStream_t s);
hipError_t dslash_tw_launch_f16_d1(const DslashArgs &a, int lk, int nr, int epi, int block, int grid, hipStream_t s);

hipError_t dslash_tw_launch(const DslashArgs &a, int sp, int lk, int nr, int dag, int epi, int block, int grid,
                            hipStream_t s)
{
    if (sp == SP_F16) return dag ? dslash_tw_launch_f16_d1(a, lk, nr, epi, block, grid, s)
                         : dslash_tw_launch_f16_d0(a, lk, nr, epi, block, grid, s);
    return hipErrorInvalidValue;
}

bool dslash_tw_supported(int sp, int lk, int nr)
{
    return sp == SP_F16 && (lk == LK_F32_12 || lk == LK_F16_12) && nr >= 1 && nr <= 3;
}

hipError_t dslash_lds_launch(const DslashArgs &a, int sp, int lk, int nr, int dag, int epi, int grid,
                             unsigned lds_bytes, hipStream_t s)
{
    if (sp == SP_F16) return dag ? dslash_lds_launch_f16_d1(a, lk, nr, epi, grid, lds_bytes, s)
                         : dslash_lds_launch_f16_d0(a, lk, nr, epi, grid, lds_bytes, s);
    if (sp == SP_F32) return dag ? dslash_lds_launch_f32_d1(a, lk, nr, epi, grid, lds_bytes, s)
                         : dslash_lds_launch_f32_d0(a, lk, nr, epi, grid, lds_bytes, s);
    return hipErrorInvalidValue;
}

bool dslash_lds_supported(int sp, int lk, int nr)
{
    if (sp == SP_F16) return (lk == LK_F32_12 || lk == LK_F16_12) && (nr == 1 || nr == 2);
    if (sp == SP_F32) return lk == LK_F32_12 && nr == 1;
    return false;
}

hipError_t dslash_launch(const DslashArgs &a, int sp, int lk, int nr, int rl, int dag, int epi, int block,
                         int grid, hipStream_t s)
{
    if (sp == SP_F64) return dag ? dslash_launch_f64_d1(a, lk, nr, rl, epi, block, grid, s)
                         : dslash_launch_f64_d0(a, lk, nr, rl, epi, block, grid, s);
    if (sp == SP_F32) return dag ? dslash_launch_f32_d1(a, lk, nr, rl, epi, block, grid, s)
                         : dslash_launch_f32_d0(a, lk, nr, rl, epi, block, grid, s);
    if (sp == SP_F16) return dag ? dslash_launch_f16_d1(a, lk, nr, rl, epi, block, grid, s)
                         : dslash_launch_f16_d0(a, lk, nr, rl, epi, block, grid, s);
    if (sp == SP_I16) return dag ? dslash_launch_i16_d1(a, lk, nr, rl, epi, block, grid, s)
                         : dslash_launch_i16_d0(a, lk, nr, rl, epi, block, grid, s);
    return hipErrorInvalidValue;
}

bool dslash_shape_supported(int sp, int lk, int nr, int rl)
{
    if (rl != 1 && rl != 2 && rl != 4) return false;
    if (lk == LK_F32_12N || lk == LK_F32_8N) return (sp == SP_F16 || sp == SP_F32) && rl == 1 && (nr == 1 || nr == 2);
    if (lk == LK_F64_12N) return sp == SP_F64 && rl == 1 && (nr == 1 || nr == 2);
    if (sp == SP_F64 || lk == LK_F32_8) return nr == 1 || nr == 2;  // (8-real links: for few RHS)
    return nr >= 1 && nr <= 4;
}

}  // namespace wd
