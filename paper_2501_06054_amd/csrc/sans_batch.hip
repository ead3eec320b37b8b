// sans_batch.hip -- the persistent kernel of the batched launch (every
// model's per-neutron code behind one scalar switch per tile).
#include "sans_kernels.hpp"

namespace sans {

namespace {

__global__ __launch_bounds__(kHistBlock) void k_batch(const TraceArgs* __restrict__ exps,
                                                      const BatchTile* __restrict__ tiles, int ntiles,
                                                      unsigned* counter, double* dets, int npix, int M)
{
    extern __shared__ double lds_d[];
    double* hist = lds_d;
    __shared__ int s_tile;
    for (;;) {
        if (threadIdx.x == 0) s_tile = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int ti = s_tile;
        if (ti >= ntiles) break;
        const BatchTile tl = tiles[ti];
        const unsigned e = __builtin_amdgcn_readfirstlane(tl.e);
        ConstArgs* a = (ConstArgs*)(exps + e);
        for (int i = threadIdx.x; i < npix; i += blockDim.x) hist[i] = 0.0;
        // the Schulz table stays in global memory (L2/L1): the histogram
        // takes the workgroup's LDS
        const double* tab = a->tab_size;
        __syncthreads();
        switch (a->kind) {
        case 0: batch_tile<0>(a, tl.first, tl.count, hist, tab); break;
        case 1: batch_tile<1>(a, tl.first, tl.count, hist, tab); break;
        case 2: batch_tile<2>(a, tl.first, tl.count, hist, tab); break;
        case 3: batch_tile<3>(a, tl.first, tl.count, hist, tab); break;
        case 4: batch_tile<4>(a, tl.first, tl.count, hist, tab); break;
        case 5: batch_tile<5>(a, tl.first, tl.count, hist, tab); break;
        case 6: batch_tile<6>(a, tl.first, tl.count, hist, tab); break;
        case 7: batch_tile<7>(a, tl.first, tl.count, hist, tab); break;
        case 8: batch_tile<8>(a, tl.first, tl.count, hist, tab); break;
        case 9: batch_tile<9>(a, tl.first, tl.count, hist, tab); break;
        case 10: batch_tile<10>(a, tl.first, tl.count, hist, tab); break;
        case 11: batch_tile<11>(a, tl.first, tl.count, hist, tab); break;
        case 12: batch_tile<12>(a, tl.first, tl.count, hist, tab); break;
        case 13: batch_tile<13>(a, tl.first, tl.count, hist, tab); break;
        case 14: batch_tile<14>(a, tl.first, tl.count, hist, tab); break;
        case 15: batch_tile<15>(a, tl.first, tl.count, hist, tab); break;
        case 16: batch_tile<16>(a, tl.first, tl.count, hist, tab); break;
        case 17: batch_tile<17>(a, tl.first, tl.count, hist, tab); break;
        case 18: batch_tile<18>(a, tl.first, tl.count, hist, tab); break;
        case 19: batch_tile<19>(a, tl.first, tl.count, hist, tab); break;
        case 20: batch_tile<20>(a, tl.first, tl.count, hist, tab); break;
        case 21: batch_tile<21>(a, tl.first, tl.count, hist, tab); break;
        case 22: batch_tile<22>(a, tl.first, tl.count, hist, tab); break;
        case 23: batch_tile<23>(a, tl.first, tl.count, hist, tab); break;
        case 24: batch_tile<24>(a, tl.first, tl.count, hist, tab); break;
        case 25: batch_tile<25>(a, tl.first, tl.count, hist, tab); break;
        case 26: batch_tile<26>(a, tl.first, tl.count, hist, tab); break;
        case 27: batch_tile<27>(a, tl.first, tl.count, hist, tab); break;
        case 28: batch_tile<28>(a, tl.first, tl.count, hist, tab); break;
        case 29: batch_tile<29>(a, tl.first, tl.count, hist, tab); break;
        case 30: batch_tile<30>(a, tl.first, tl.count, hist, tab); break;
        case 31: batch_tile<31>(a, tl.first, tl.count, hist, tab); break;
        case 32: batch_tile<32>(a, tl.first, tl.count, hist, tab); break;
        case 33: batch_tile<33>(a, tl.first, tl.count, hist, tab); break;
        case 34: batch_tile<34>(a, tl.first, tl.count, hist, tab); break;
        case 35: batch_tile<35>(a, tl.first, tl.count, hist, tab); break;
        case 36: batch_tile<36>(a, tl.first, tl.count, hist, tab); break;
        case 37: batch_tile<37>(a, tl.first, tl.count, hist, tab); break;
        case 38: batch_tile<38>(a, tl.first, tl.count, hist, tab); break;
        case 39: batch_tile<39>(a, tl.first, tl.count, hist, tab); break;
        case 40: batch_tile<40>(a, tl.first, tl.count, hist, tab); break;
        case 41: batch_tile<41>(a, tl.first, tl.count, hist, tab); break;
        case 42: batch_tile<42>(a, tl.first, tl.count, hist, tab); break;
        case 43: batch_tile<43>(a, tl.first, tl.count, hist, tab); break;
        case 44: batch_tile<44>(a, tl.first, tl.count, hist, tab); break;
        case 45: batch_tile<45>(a, tl.first, tl.count, hist, tab); break;
        case 46: batch_tile<46>(a, tl.first, tl.count, hist, tab); break;
        case 47: batch_tile<47>(a, tl.first, tl.count, hist, tab); break;
        case 48: batch_tile<48>(a, tl.first, tl.count, hist, tab); break;
        case 49: batch_tile<49>(a, tl.first, tl.count, hist, tab); break;
        case 50: batch_tile<50>(a, tl.first, tl.count, hist, tab); break;
        case 51: batch_tile<51>(a, tl.first, tl.count, hist, tab); break;
        case 52: batch_tile<52>(a, tl.first, tl.count, hist, tab); break;
        case 53: batch_tile<53>(a, tl.first, tl.count, hist, tab); break;
        case 54: batch_tile<54>(a, tl.first, tl.count, hist, tab); break;
        case 55: batch_tile<55>(a, tl.first, tl.count, hist, tab); break;
        case 56: batch_tile<56>(a, tl.first, tl.count, hist, tab); break;
        case 57: batch_tile<57>(a, tl.first, tl.count, hist, tab); break;
        case 58: batch_tile<58>(a, tl.first, tl.count, hist, tab); break;
        case 59: batch_tile<59>(a, tl.first, tl.count, hist, tab); break;
        case 60: batch_tile<60>(a, tl.first, tl.count, hist, tab); break;
        case 61: batch_tile<61>(a, tl.first, tl.count, hist, tab); break;
        case 62: batch_tile<62>(a, tl.first, tl.count, hist, tab); break;
        default: batch_tile<63>(a, tl.first, tl.count, hist, tab); break;
        }
        __syncthreads();
        double* det = dets + (size_t)e * npix;
        for (int i = threadIdx.x; i < npix; i += blockDim.x) {
            const double v = hist[i];
            if (v != 0.0) __hip_atomic_fetch_add(det + i, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        __syncthreads();
    }
}

}  // namespace

BatchFn batch_kernel() { return k_batch; }

}  // namespace sans
