// Launchers of the pruned pipeline for every supported P, with the per-plan
// kernel variant; instantiated per arithmetic by the launch_pruned_*.hip units.
#pragma once
#include "k_pruned.hpp"
#include "ps_internal.hpp"

namespace ps {

template <typename T> struct PrunedShape {
    static constexpr int ZT = sizeof(T) == 4 ? 16 : 8;  // y-pass tile: 128-byte rows of interleaved pencils
    static constexpr int ZB = ZT;                       // z pass: rows of interleaved pencils too (variant
                                                        // ztile 1 halves it: 64-byte rows, half the LDS)
};

// Threads of a workgroup whose B pencils are each owned by one wavefront
// holding >= E elements per lane (several pencils per wave for short P).
constexpr int wave_threads(int B, int P, int E)
{
    int ppw = 1;  // largest power of two dividing B with ppw P <= 64 E
    while (ppw * 2 <= B && B % (ppw * 2) == 0 && ppw * 2 * P <= 64 * E) ppw *= 2;
    return 64 * (B / ppw);
}

// Whether the persistent z pass (EL elements per lane) fits the 160 KB of LDS
// a workgroup can hold: its pencil buffer plus the copy of the column twiddles.
template <typename T, int P, int FAM, int EL, int MT, int B = PrunedShape<T>::ZB> constexpr bool z_pf_fits()
{
    using TL = TileZConv<T, P, FAM, B, wave_threads(B, P, EL), true, MT>;
    using RF = typename PlanFor<P, FAM>::Fwd;
    using RI = typename PlanFor<P, FAM>::Inv;
    constexpr int C = RF::tw_size() + (std::is_same<RF, RI>::value ? 0 : RI::tw_size());
    return (TL::LDS + C) * (int)sizeof(cx<T>) <= 160 * 1024;
}

// Whether the x passes with ROWS rows per workgroup fit the LDS.
template <typename T, int P, int FAM, int ROWS, int MT> constexpr bool x_fits()
{
    constexpr int NTR = threads_for(ROWS / 2, P, FAM == 1 ? fam1_elems<P>() : 16);
    return TileXR2C<T, P, FAM, NTR, MAP_EF, MT, false, ROWS>::LDS * (int)sizeof(cx<T>) <= 160 * 1024 &&
           TileXC2R<T, P, FAM, NTR, MAP_EF, MT, false, ROWS>::LDS * (int)sizeof(cx<T>) <= 160 * 1024;
}

// Workgroups of `kernel` (nt threads) resident on the device at once, rounded
// down to a multiple of 8 (the XCD count); a fallback if the query fails.
template <class K> static int resident_workgroups(K kernel, int nt)
{
    int dev = 0, cus = 0, per_cu = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess &&
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, nt, 0) == hipSuccess && per_cu * cus >= 8)
        return per_cu * cus / 8 * 8;
    return 1024;
}

template <typename T, int P, int FAM, int MT> struct PassLaunch {
    using V = cx<T>;
    static constexpr int N = P / 2, H = N + 1;
    static constexpr int ZT = PrunedShape<T>::ZT, ZB = PrunedShape<T>::ZB;
    // elements per thread: 32 for the radix-32-based family, else 16; the
    // z pass of split plans also takes 32 (its matrix-core DFT-16 operands
    // and accumulators need the register budget of half as many threads:
    // at 16 the compiler spilled and the pass moved 1.4x its bytes)
    static constexpr int E = FAM == 1 ? fam1_elems<P>() : 16;
    static constexpr int EZ = FAM == 1 ? fam1_elems<P>() : MT > 0 ? 32 : 16;
    static constexpr int NTX = threads_for(8, P, E);
    static constexpr int NTY = threads_for(ZT, P, E);

    // x passes: ROWS rows of one z-plane per workgroup (ROWS / 2 packed pencils)
    template <int ROWS = 16> static void x_r2c(const PrunedBufs& b)
    {
        constexpr int NTR = threads_for(ROWS / 2, P, E);
        hipLaunchKernelGGL((k_x_r2c<T, P, FAM, NTR, MAP_EF, MT, false, ROWS>), dim3((N + ROWS - 1) / ROWS, N, b.count),
                           dim3(NTR), 0, b.stream, static_cast<const T*>(b.in[0]), static_cast<V*>(b.out[0]), b.list,
                           b.stab);
    }
    // y passes: Z pencils per workgroup (the full tile ZT or half of it)
    // (HALF: stage exchanges through half the LDS in two rounds)
    template <int Z = ZT, bool HALF = false> static void y_fwd(const PrunedBufs& b)
    {
        constexpr int NTZY = threads_for(Z, P, E);
        hipLaunchKernelGGL((k_y_fwd<T, P, FAM, Z, NTZY, MAP_EF, MT, false, HALF>), dim3((N + Z - 1) / Z, H, b.count), dim3(NTZY),
                           0, b.stream, static_cast<const V*>(b.in[1]), static_cast<V*>(b.out[1]), b.list, b.stab);
    }
    // z pass: B pencils per workgroup (the full tile ZB or half of it)
    template <bool WAVE, int B = ZB> static void z_conv(const PrunedBufs& b)
    {
        constexpr int NTZ = WAVE ? wave_threads(B, P, EZ) : threads_for(B, P, EZ);
        hipLaunchKernelGGL((k_z_conv<T, P, FAM, B, NTZ, WAVE, MT>), dim3(P / B, H, b.count), dim3(NTZ), 0, b.stream,
                           static_cast<const V*>(b.in[2]), static_cast<V*>(b.out[2]), b.list, b.stab);
    }
    // z pass exchanging through half the LDS in two rounds (wave-owned pencils)
    template <int B = ZB> static void z_conv_half(const PrunedBufs& b)
    {
        constexpr int NTZ = wave_threads(B, P, EZ);
        hipLaunchKernelGGL((k_z_conv_half<T, P, FAM, B, NTZ>), dim3(P / B, H, b.count), dim3(NTZ), 0, b.stream,
                           static_cast<const V*>(b.in[2]), static_cast<V*>(b.out[2]), b.list, b.stab);
    }
    // Persistent passes: as many workgroups as fit on the device at once (a
    // multiple of 8, so z tile pairs stay on one XCD), each walking tiles.
    // EL: elements per lane that set the pencils per wavefront (32: two or
    // more 1024-point pencils per wavefront, 16: one).
    template <int EL, int B = ZB> static void z_conv_pf(const PrunedBufs& b)
    {
        constexpr int NTZ = wave_threads(B, P, EL);
        static const int resident = resident_workgroups(k_z_conv_pf<T, P, FAM, B, NTZ, MT>, NTZ);
        const int total = (P / B) * H * b.count;
        hipLaunchKernelGGL((k_z_conv_pf<T, P, FAM, B, NTZ, MT>), dim3(total < resident ? total : resident),
                           dim3(NTZ), 0, b.stream, static_cast<const V*>(b.in[2]), static_cast<V*>(b.out[2]), b.list,
                           b.stab, b.count);
    }
    static void y_fwd_pf(const PrunedBufs& b)
    {
        static const int resident = resident_workgroups(k_y_fwd_pf<T, P, FAM, ZT, NTY, MT>, NTY);
        const int total = ((N + ZT - 1) / ZT) * H * b.count;
        hipLaunchKernelGGL((k_y_fwd_pf<T, P, FAM, ZT, NTY, MT>), dim3(total < resident ? total : resident), dim3(NTY),
                           0, b.stream, static_cast<const V*>(b.in[1]), static_cast<V*>(b.out[1]), b.list, b.stab,
                           b.count);
    }
    static void y_inv_pf(const PrunedBufs& b)
    {
        static const int resident = resident_workgroups(k_y_inv_pf<T, P, FAM, ZT, NTY, MT>, NTY);
        const int total = ((H + ZT - 1) / ZT) * N * b.count;
        hipLaunchKernelGGL((k_y_inv_pf<T, P, FAM, ZT, NTY, MT>), dim3(total < resident ? total : resident), dim3(NTY),
                           0, b.stream, static_cast<const V*>(b.in[3]), static_cast<V*>(b.out[3]), b.list, b.stab,
                           b.count);
    }
    template <int Z = ZT, bool HALF = false> static void y_inv(const PrunedBufs& b)
    {
        constexpr int NTZY = threads_for(Z, P, E);
        hipLaunchKernelGGL((k_y_inv<T, P, FAM, Z, NTZY, MAP_EF, MT, false, HALF>), dim3((H + Z - 1) / Z, N, b.count), dim3(NTZY),
                           0, b.stream, static_cast<const V*>(b.in[3]), static_cast<V*>(b.out[3]), b.list, b.stab);
    }
    template <int ROWS = 16> static void x_c2r(const PrunedBufs& b)
    {
        constexpr int NTR = threads_for(ROWS / 2, P, E);
        hipLaunchKernelGGL((k_x_c2r<T, P, FAM, NTR, MAP_EF, MT, false, ROWS>), dim3((N + ROWS - 1) / ROWS, N, b.count),
                           dim3(NTR), 0, b.stream, static_cast<const V*>(b.in[4]), static_cast<T*>(b.out[4]), b.list,
                           b.stab);
    }

    // Box forms: P is the transformed axis's length; the grids cover the
    // other two axes' extents b.nx, b.ny, b.nz (the kernels read them from
    // the solve records, so every record of a launch has the same box).
    static void x_r2c_box(const PrunedBufs& b)
    {
        hipLaunchKernelGGL((k_x_r2c<T, P, FAM, NTX, MAP_EF, MT, true>), dim3((b.ny + 15) / 16, b.nz, b.count),
                           dim3(NTX), 0, b.stream, static_cast<const T*>(b.in[0]), static_cast<V*>(b.out[0]), b.list,
                           b.stab);
    }
    static void y_fwd_box(const PrunedBufs& b)
    {
        hipLaunchKernelGGL((k_y_fwd<T, P, FAM, ZT, NTY, MAP_EF, MT, true>),
                           dim3((b.nz + ZT - 1) / ZT, b.nx + 1, b.count), dim3(NTY), 0, b.stream,
                           static_cast<const V*>(b.in[1]), static_cast<V*>(b.out[1]), b.list, b.stab);
    }
    template <bool WAVE, int B = ZB> static void z_conv_box(const PrunedBufs& b)
    {
        constexpr int NTZ = WAVE ? wave_threads(B, P, EZ) : threads_for(B, P, EZ);
        hipLaunchKernelGGL((k_z_conv<T, P, FAM, B, NTZ, WAVE, MT, true>), dim3(2 * b.ny / B, b.nx + 1, b.count),
                           dim3(NTZ), 0, b.stream, static_cast<const V*>(b.in[2]), static_cast<V*>(b.out[2]), b.list,
                           b.stab);
    }
    static void y_inv_box(const PrunedBufs& b)
    {
        hipLaunchKernelGGL((k_y_inv<T, P, FAM, ZT, NTY, MAP_EF, MT, true>),
                           dim3((b.nx + 1 + ZT - 1) / ZT, b.nz, b.count), dim3(NTY), 0, b.stream,
                           static_cast<const V*>(b.in[3]), static_cast<V*>(b.out[3]), b.list, b.stab);
    }
    static void x_c2r_box(const PrunedBufs& b)
    {
        hipLaunchKernelGGL((k_x_c2r<T, P, FAM, NTX, MAP_EF, MT, true>), dim3((b.ny + 15) / 16, b.nz, b.count),
                           dim3(NTX), 0, b.stream, static_cast<const V*>(b.in[4]), static_cast<T*>(b.out[4]), b.list,
                           b.stab);
    }
};

// The z pass of a box with B pencils per workgroup.
template <typename T, int P, int MT, int B> static void box_z(int zmode, const PrunedBufs& b)
{
    using L0 = PassLaunch<T, P, 0, MT>;
    constexpr bool F1 = has_fam1<P>() && MT == 0;
    using L1 = PassLaunch<T, P, F1 ? 1 : 0, MT>;
    if (zmode == 2 && F1) L1::template z_conv_box<true, B>(b);
    else if (zmode >= 1) L0::template z_conv_box<true, B>(b);
    else L0::template z_conv_box<false, B>(b);
}

// One pass of a box solve with P its axis's length.  Boxes run the
// one-tile-per-workgroup kernels (persistent variants are for cubes).
template <typename T, int P, int MT> static hipError_t box_pass(int pass, const PrunedBufs& b)
{
    using L0 = PassLaunch<T, P, 0, MT>;
    constexpr bool F1 = has_fam1<P>() && MT == 0;
    using L1 = PassLaunch<T, P, F1 ? 1 : 0, MT>;
    const PrunedVariant& v = b.var;
    switch (pass) {
    case 0:
        if (v.x_fam >> 1) return hipErrorInvalidValue;  // boxes: 16 rows per x tile
        if (v.x_fam == 1 && F1) L1::x_r2c_box(b);
        else L0::x_r2c_box(b);
        break;
    case 1:
        if (v.y_fam & 6) return hipErrorInvalidValue;  // boxes: one tile per workgroup, full tile
        if ((v.y_fam & 1) && F1) L1::y_fwd_box(b);
        else L0::y_fwd_box(b);
        break;
    case 2:
        if (v.zmode >= 3) return hipErrorInvalidValue;
        if (v.ztile == 1) box_z<T, P, MT, PrunedShape<T>::ZB / 2>(v.zmode, b);
        else box_z<T, P, MT, PrunedShape<T>::ZB>(v.zmode, b);
        break;
    case 3:
        if (v.yi_fam & 6) return hipErrorInvalidValue;
        if ((v.yi_fam & 1) && F1) L1::y_inv_box(b);
        else L0::y_inv_box(b);
        break;
    case 4:
        if (v.xc_fam >> 1) return hipErrorInvalidValue;
        if (v.xc_fam == 1 && F1) L1::x_c2r_box(b);
        else L0::x_c2r_box(b);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

// An x pass of a cube: variant = family (bit 0) + 2 x rows selector (0: 16
// rows per workgroup, 1: 8, 2: 32).  False for a tile the LDS cannot hold.
template <typename T, int P, int MT, int ROWS> static bool x_rows(bool inverse, bool fam1, const PrunedBufs& b)
{
    constexpr bool F1 = has_fam1<P>() && MT == 0;
    using L0 = PassLaunch<T, P, 0, MT>;
    using L1 = PassLaunch<T, P, F1 ? 1 : 0, MT>;
    if (fam1 && F1) {
        if constexpr (x_fits<T, P, F1 ? 1 : 0, ROWS, MT>()) {
            if (inverse) L1::template x_c2r<ROWS>(b);
            else L1::template x_r2c<ROWS>(b);
            return true;
        }
        return false;
    }
    if constexpr (x_fits<T, P, 0, ROWS, MT>()) {
        if (inverse) L0::template x_c2r<ROWS>(b);
        else L0::template x_r2c<ROWS>(b);
        return true;
    }
    return false;
}
template <typename T, int P, int MT> static bool x_pass(bool inverse, int variant, const PrunedBufs& b)
{
    const bool fam1 = variant & 1;
    switch (variant >> 1) {
    case 0: return x_rows<T, P, MT, 16>(inverse, fam1, b);
    case 1: return x_rows<T, P, MT, 8>(inverse, fam1, b);
    case 2: return x_rows<T, P, MT, 32>(inverse, fam1, b);
    default: return false;
    }
}

// The fused z pass of a cube with B pencils per workgroup, in form zmode.
template <typename T, int P, int MT, int B> static void cube_z(int zmode, const PrunedBufs& b)
{
    using L0 = PassLaunch<T, P, 0, MT>;
    constexpr bool F1 = has_fam1<P>() && MT == 0;
    using L1 = PassLaunch<T, P, F1 ? 1 : 0, MT>;
    if constexpr (PlanFor<P, F1 ? 1 : 0>::Fwd::S > 1 && z_pf_fits<T, P, F1 ? 1 : 0, 32, MT, B>()) {
        if (zmode == 3) {  // persistent: radix-32 family where it exists
            L1::template z_conv_pf<32, B>(b);
            return;
        }
    }
    if constexpr (PlanFor<P, 0>::Fwd::S > 1 && z_pf_fits<T, P, 0, 16, MT, B>()) {
        if (zmode == 4) {  // persistent: radix-16 family, one 1024-point pencil per wavefront
            L0::template z_conv_pf<16, B>(b);
            return;
        }
    }
    if constexpr (P >= 512 && F1) {
        if (zmode == 5) {  // half-LDS exchange on the two-stage plan
            L1::template z_conv_half<B>(b);
            return;
        }
    }
    // (a persistent form that does not fit runs as the wave-owned pass of its own family)
    if ((zmode == 2 || zmode == 3) && F1) L1::template z_conv<true, B>(b);
    else if (zmode >= 1) L0::template z_conv<true, B>(b);
    else L0::template z_conv<false, B>(b);
}

// Split matrix-core plans keep the radix-16 family (family 1 has no radix-16 stage).
template <typename T, int P, int MT> static hipError_t pruned_passes(int lo, int hi, const PrunedBufs& b)
{
    using L0 = PassLaunch<T, P, 0, MT>;
    constexpr bool F1 = has_fam1<P>() && MT == 0;
    using L1 = PassLaunch<T, P, F1 ? 1 : 0, MT>;
    const PrunedVariant& v = b.var;
    for (int pass = lo; pass < hi; ++pass) {
        switch (pass) {
        case 0:
            if (!x_pass<T, P, MT>(false, v.x_fam, b)) return hipErrorInvalidValue;
            break;
        case 1:
            // variant bit 0: two-stage family, bit 1: persistent, 4 and 5: half
            // tile, 6 and 7: stage exchanges through half the LDS
            if (v.y_fam >= 6) {
                if constexpr (P >= 512 && MT == 0) {
                    if ((v.y_fam & 1) && F1) L1::template y_fwd<PrunedShape<T>::ZT, true>(b);
                    else L0::template y_fwd<PrunedShape<T>::ZT, true>(b);
                } else {
                    return hipErrorInvalidValue;
                }
            } else if (v.y_fam >= 4) {
                if ((v.y_fam & 1) && F1) L1::template y_fwd<PrunedShape<T>::ZT / 2>(b);
                else L0::template y_fwd<PrunedShape<T>::ZT / 2>(b);
            } else if ((v.y_fam & 1) && F1) (v.y_fam & 2) ? L1::y_fwd_pf(b) : L1::y_fwd(b);
            else (v.y_fam & 2) ? L0::y_fwd_pf(b) : L0::y_fwd(b);
            break;
        case 2:
            if (v.ztile == 1) cube_z<T, P, MT, PrunedShape<T>::ZB / 2>(v.zmode, b);
            else cube_z<T, P, MT, PrunedShape<T>::ZB>(v.zmode, b);
            break;
        case 3:
            if (v.yi_fam >= 6) {
                if constexpr (P >= 512 && MT == 0) {
                    if ((v.yi_fam & 1) && F1) L1::template y_inv<PrunedShape<T>::ZT, true>(b);
                    else L0::template y_inv<PrunedShape<T>::ZT, true>(b);
                } else {
                    return hipErrorInvalidValue;
                }
            } else if (v.yi_fam >= 4) {
                if ((v.yi_fam & 1) && F1) L1::template y_inv<PrunedShape<T>::ZT / 2>(b);
                else L0::template y_inv<PrunedShape<T>::ZT / 2>(b);
            } else if ((v.yi_fam & 1) && F1) (v.yi_fam & 2) ? L1::y_inv_pf(b) : L1::y_inv(b);
            else (v.yi_fam & 2) ? L0::y_inv_pf(b) : L0::y_inv(b);
            break;
        case 4:
            if (!x_pass<T, P, MT>(true, v.xc_fam, b)) return hipErrorInvalidValue;
            break;
        default:
            return hipErrorInvalidValue;
        }
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// Passes [lo, hi): a cube's run on its one length; a box's each on the
// length of the axis it transforms (x: passes 0 and 4, y: 1 and 3, z: 2).
// Only the lengths of one half (is_short_p(P) == SHORT) are instantiated
// here, so that each arithmetic compiles as two units in parallel; the
// other half returns hipErrorInvalidValue (pruned_run in ps_internal.hpp
// routes every pass to its half).
template <typename T, int MT, bool SHORT> static hipError_t pruned_dispatch(int lo, int hi, const PrunedBufs& b)
{
    if (!b.box) {
        switch (b.px) {
#define PS_CASE(PP)                                                           \
    case PP:                                                                  \
        if constexpr (is_short_p(PP) == SHORT) return pruned_passes<T, PP, MT>(lo, hi, b); \
        else return hipErrorInvalidValue;
            PS_FOR_EACH_P(PS_CASE)
#undef PS_CASE
        default: return hipErrorInvalidValue;
        }
    }
    for (int pass = lo; pass < hi; ++pass) {
        const int P = pass == 2 ? b.pz : (pass == 1 || pass == 3) ? b.py : b.px;
        hipError_t e = hipErrorInvalidValue;
        switch (P) {
#define PS_CASE(PP)                                                           \
    case PP:                                                                  \
        if constexpr (is_short_p(PP) == SHORT) e = box_pass<T, PP, MT>(pass, b); \
        break;
            PS_FOR_EACH_P(PS_CASE)
#undef PS_CASE
        default: break;
        }
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

}  // namespace ps
