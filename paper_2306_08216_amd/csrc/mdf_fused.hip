// Dispatch of the fused single-pass step (one wave per 64 lanes of a strip)
// to the kernel families of mdf_fused_impl.hpp, instantiated per tile width
// and fluid model in mdf_fused_w*.hip.
#include "mdf_fused_impl.hpp"

namespace mdf {

#define MDF_FAMILY_DECL(TW, PLW)                                                                                     \
    extern template hipError_t launch_fused_family<TW, PLW>(const StepConsts&, const fusedk::FusedGrid&, int,          \
                                                            const double*, double*, hipStream_t);                    \
    extern template hipError_t launch_batch_family<TW, PLW>(const BatchInst*, const int4*, int, int, int,              \
                                                            const double*, double*, hipStream_t);
MDF_FAMILY_DECL(64, false)
MDF_FAMILY_DECL(64, true)
MDF_FAMILY_DECL(128, false)
MDF_FAMILY_DECL(128, true)
MDF_FAMILY_DECL(256, false)
MDF_FAMILY_DECL(256, true)
#undef MDF_FAMILY_DECL

bool fused_shape_ok(const StepConsts& K, FusedShape sh)
{
    if (K.ff) return sh.tile_w == 64 && sh.prefetch == 2;   // force-field kernels: 64 lanes, prefetch 2
    return (sh.tile_w == 64 || sh.tile_w == 128 || sh.tile_w == 256) && sh.prefetch >= 2 && sh.prefetch <= 3;
}

hipError_t launch_fused_batch(const BatchInst* insts, const int4* table, int nwg, int pl, int tile_w, int prefetch,
                              const double* fin, double* fout, hipStream_t s)
{
    if (nwg <= 0) return hipErrorInvalidValue;
    const bool law = pl != PL_NEWTON;
    switch (tile_w) {
    case 64:
        return law ? launch_batch_family<64, true>(insts, table, nwg, pl, prefetch, fin, fout, s)
                   : launch_batch_family<64, false>(insts, table, nwg, pl, prefetch, fin, fout, s);
    case 128:
        return law ? launch_batch_family<128, true>(insts, table, nwg, pl, prefetch, fin, fout, s)
                   : launch_batch_family<128, false>(insts, table, nwg, pl, prefetch, fin, fout, s);
    case 256:
        return law ? launch_batch_family<256, true>(insts, table, nwg, pl, prefetch, fin, fout, s)
                   : launch_batch_family<256, false>(insts, table, nwg, pl, prefetch, fin, fout, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t launch_fused(const StepConsts& K, FusedShape sh, const double* fin, double* fout, hipStream_t s)
{
    fusedk::FusedGrid G;
    const int wout = sh.tile_w - 8;
    const bool tasks = sh.wall_tasks && sh.seg_h <= 0;
    G.xoff = tasks ? kWallCols : 0;
    G.xspan = tasks ? K.nx - 2 * kWallCols : K.nx;
    G.nstrips = (G.xspan + wout - 1) / wout;
    if (sh.seg_h > 0) {
        G.nsegs = (K.ny + sh.seg_h - 1) / sh.seg_h;
        G.nwg = G.nstrips * G.nsegs;
        G.table = nullptr;
    } else {
        if (!sh.table || sh.nwg <= 0) return hipErrorInvalidValue;
        G.nsegs = 0;
        G.nwg = sh.nwg;
        G.table = sh.table;
    }
    G.chunk = (G.nwg + 7) / 8;
    const bool pl = K.pl != PL_NEWTON;
    switch (sh.tile_w) {
    case 64:
        return pl ? launch_fused_family<64, true>(K, G, sh.prefetch, fin, fout, s)
                  : launch_fused_family<64, false>(K, G, sh.prefetch, fin, fout, s);
    case 128:
        return pl ? launch_fused_family<128, true>(K, G, sh.prefetch, fin, fout, s)
                  : launch_fused_family<128, false>(K, G, sh.prefetch, fin, fout, s);
    case 256:
        return pl ? launch_fused_family<256, true>(K, G, sh.prefetch, fin, fout, s)
                  : launch_fused_family<256, false>(K, G, sh.prefetch, fin, fout, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace mdf
