// Persistent batched solves: many independent solves of uneven sizes in one
// launch.  The paper runs one nested-mesh level per GPU and notes that
// streams could split a GPU among several levels (section 3); here a single
// persistent kernel drains a work list of (solve, pass, tile) items instead.
//
// Work list.  Items are ordered pass-major: every x_r2c tile of every solve,
// then every y_fwd tile, and so on; within a pass the solves keep the order
// the host gave them (largest first).  Workgroups take the next item from an
// atomic counter, so uneven sizes balance dynamically.  Before a tile of pass
// k > 0 of solve i runs, the workgroup waits until all tiles of pass k - 1 of
// solve i have completed (a per-(solve, pass) counter, released at agent
// scope after the tile's stores, acquired before the dependent tile's loads).
// A workgroup only ever waits for items handed out before its own, and those
// are held by running workgroups, so the wait always ends; it is still
// bounded by a spin limit, after which the kernel records an error flag and
// skips the tile instead of hanging.
#pragma once
#include "batch_types.hpp"
#include "k_pruned.hpp"

namespace ps {

template <typename T, int P, int NT, int MT> struct BatchTiles {
    static constexpr int ZT = sizeof(T) == 4 ? 16 : 8;
    using TX = TileXR2C<T, P, 0, NT, MAP_EF, MT>;
    using TY = TileYFwd<T, P, 0, ZT, NT, MAP_EF, MT>;
    using TZ = TileZConv<T, P, 0, ZT, NT, true, MT>;
    using TI = TileYInv<T, P, 0, ZT, NT, MAP_EF, MT>;
    using TC = TileXC2R<T, P, 0, NT, MAP_EF, MT>;
    static constexpr int m2(int a, int b) { return a > b ? a : b; }
    static constexpr int LDS = m2(m2(m2(TX::LDS, TY::LDS), m2(TZ::LDS, TI::LDS)), TC::LDS);

    // Not inlined: each length gets its own register allocation instead of
    // one allocation for the union of all lengths.
    __device__ __noinline__ static void run(const BatchSolve& s, int pass, int tile, cx<T>* lds,
                                            const SplitA<MT>& sa)
    {
        using V = cx<T>;
        constexpr int N = P / 2;
        const V* twf = static_cast<const V*>(s.twf);
        const V* twi = static_cast<const V*>(s.twi);
        switch (pass) {
        case 0: {
            constexpr int nx = (N + 15) / 16;
            TX::run(tile % nx, tile / nx, static_cast<const T*>(s.rho), static_cast<V*>(s.t1), twf, lds, sa);
            break;
        }
        case 1: {
            constexpr int nz = (N + ZT - 1) / ZT;
            TY::run(tile % nz, tile / nz, static_cast<const V*>(s.t1), static_cast<V*>(s.t2), twf, lds, sa);
            break;
        }
        case 2: {
            constexpr int nq = P / ZT;
            TZ::run(tile % nq, tile / nq, static_cast<const V*>(s.t2), static_cast<V*>(s.t3),
                    static_cast<const T*>(s.ghat), twf, twi, lds, sa);
            break;
        }
        case 3: {
            constexpr int nk = (N + 1 + ZT - 1) / ZT;
            TI::run(tile % nk, tile / nk, static_cast<const V*>(s.t3), static_cast<V*>(s.t1), twi, lds, sa);
            break;
        }
        default: {
            constexpr int nx = (N + 15) / 16;
            TC::run(tile % nx, tile / nx, static_cast<const V*>(s.t1), static_cast<T*>(s.phi), twi, lds, sa);
            break;
        }
        }
    }
};

// Sizes compiled into a persistent kernel whose largest length is PMAX.
template <int PMAX> struct BatchSizes;
template <> struct BatchSizes<256> {
    static constexpr int n = 8;
    static constexpr int p[8] = {16, 32, 48, 64, 96, 128, 192, 256};
};
template <> struct BatchSizes<1024> {
    static constexpr int n = 12;
    static constexpr int p[12] = {16, 32, 48, 64, 96, 128, 192, 256, 384, 512, 768, 1024};
};

template <typename T, int PMAX, int NT, int MT, int K = 0> constexpr int batch_lds()
{
    if constexpr (K >= BatchSizes<PMAX>::n) {
        return 0;
    } else {
        constexpr int here = BatchTiles<T, BatchSizes<PMAX>::p[K], NT, MT>::LDS;
        constexpr int rest = batch_lds<T, PMAX, NT, MT, K + 1>();
        return here > rest ? here : rest;
    }
}

template <typename T, int PMAX, int NT, int MT, int K = 0>
__device__ __forceinline__ void batch_dispatch(const BatchSolve& s, int pass, int tile, cx<T>* lds,
                                               const SplitA<MT>& sa)
{
    if constexpr (K < BatchSizes<PMAX>::n) {
        constexpr int PP = BatchSizes<PMAX>::p[K];
        if (s.P == PP) BatchTiles<T, PP, NT, MT>::run(s, pass, tile, lds, sa);
        else batch_dispatch<T, PMAX, NT, MT, K + 1>(s, pass, tile, lds, sa);
    }
}

static __global__ void k_batch_reset(BatchCtl* ctl, unsigned* done, int n)
{
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        ctl->next = 0;
        ctl->error = 0;
    }
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) done[i] = 0;
}

template <typename T, int PMAX, int NT, int MT>
__global__ __launch_bounds__(NT) void k_batched(BatchCtl* __restrict__ ctl, const BatchSolve* __restrict__ sol,
                                                const int* __restrict__ prefix, unsigned* __restrict__ done,
                                                const unsigned short* __restrict__ stab, unsigned spin_limit)
{
    using V = cx<T>;
    __shared__ V lds[batch_lds<T, PMAX, NT, MT>()];
    __shared__ int s_item;
    SplitA<MT> sa;
    sa.load(stab);
    const int ns = ctl->nsolves;
    const int total = ctl->total;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = (int)atomicAdd(&ctl->next, 1u);
        __syncthreads();
        const int g = s_item;
        if (g >= total) break;
        int pass = 0;
        while (pass < 4 && g >= ctl->pass_begin[pass + 1]) ++pass;
        const int local = g - ctl->pass_begin[pass];
        const int* pf = prefix + pass * (ns + 1);
        int lo = 0, hi = ns;  // pf[lo] <= local < pf[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (pf[mid] <= local) lo = mid;
            else hi = mid;
        }
        const int i = lo;
        const int tile = local - pf[i];
        const BatchSolve s = sol[i];
        if (pass > 0) {
            __shared__ int s_ok;
            if (threadIdx.x == 0) {
                const unsigned need = (unsigned)s.ntile[pass - 1];
                unsigned spins = 0;
                int ok = 1;
                while (__hip_atomic_load(&done[i * 5 + pass - 1], __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < need) {
                    __builtin_amdgcn_s_sleep(1);
                    // give up at the spin limit, or at once if another wait already gave up
                    if (++spins > spin_limit ||
                        __hip_atomic_load(&ctl->error, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) {
                        __hip_atomic_store(&ctl->error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                        ok = 0;
                        break;
                    }
                }
                s_ok = ok;
            }
            __syncthreads();
            if (!s_ok) continue;
        }
        batch_dispatch<T, PMAX, NT, MT>(s, pass, tile, lds, sa);
        // make this tile's stores visible device-wide, then count it done
        __threadfence();
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(&done[i * 5 + pass], 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

}  // namespace ps
