// Configuration and helpers shared by the HIP kernel files of the diffraction path.
#pragma once
#include <cmath>
#include <cstdlib>
#include <cstddef>
#include <cstdint>
#include <map>
#include <mutex>
#include <type_traits>
#include <utility>

#include "fft_device.hpp"
#include "launch.hpp"

namespace cwo {

// ---- configuration per transform length --------------------------------------

// Row passes: one transform per thread group of T = M/E threads, RPB rows per block.
template <int M>
struct RowCfg {
    static constexpr int E = 16;
    static constexpr int T = M / E;
    static constexpr int RPB = (T >= 256) ? 1 : 256 / T;  // rows per block
    static constexpr int THREADS = T * RPB;
};

// Column pass: each thread transforms two adjacent columns (16-byte loads and
// stores, one 16-byte LDS slot per element pair); PAIRS column pairs per block.
template <int M>
struct ColCfg {
    // 16 values per thread at every length (T = M/16 threads per column pair, up to 512
    // at M = 8192, whose two columns then take 139 KB of LDS: one block per CU)
    static constexpr int E = 16;
    static constexpr int T = M / E;
    // two adjacent columns per thread: 16-byte accesses, shared twiddles
    static constexpr int P = 2;
    static constexpr bool SPLIT = false;
    static constexpr int LDS_PAIR = (SPLIT ? 1 : P) * lds_elems<M>();  // float2 entries per pair
    static constexpr int BY_THR = (T >= 256) ? 1 : 256 / T;
    static constexpr int BY_LDS0 = (72 * 1024) / (LDS_PAIR * 8);
    static constexpr int BY_LDS = BY_LDS0 < 1 ? 1 : BY_LDS0;
    static constexpr int PAIRS0 = BY_THR < BY_LDS ? BY_THR : BY_LDS;
    static constexpr int PAIRS = PAIRS0 > 16 ? 16 : PAIRS0;
    static constexpr int THREADS = T * PAIRS;
    static constexpr int COLS = P * PAIRS;  // columns per block
    static constexpr int WAVES_PER_EU = 2;
};

// z-stack column pass: the forward spectrum stays in registers while each plane's
// inverse transform runs on a copy, so one column per thread.
template <int M>
struct ZColCfg {
    static constexpr int E = 16;
    static constexpr int T = M / E;
    static constexpr int P = 1;
    static constexpr int LDS_PAIR = lds_elems<M>();
    static constexpr int BY_THR = (T >= 256) ? 1 : 256 / T;
    static constexpr int BY_LDS0 = (72 * 1024) / (LDS_PAIR * 8);
    static constexpr int BY_LDS = BY_LDS0 < 1 ? 1 : BY_LDS0;
    static constexpr int PAIRS0 = BY_THR < BY_LDS ? BY_THR : BY_LDS;
    static constexpr int PAIRS = PAIRS0 > 16 ? 16 : PAIRS0;
    static constexpr int THREADS = T * PAIRS;
    static constexpr int COLS = P * PAIRS;
};

// Consecutive workgroup ids are dispatched round-robin over the 8 XCDs, which
// have separate L2 caches. Remap so that each XCD works on a contiguous range
// of tiles; neighbouring tiles share cache lines.
__device__ __forceinline__ int xcd_remap(int bid, int nblocks) {
    if ((nblocks & 7) != 0) return bid;
    const int per = nblocks >> 3;
    return (bid & 7) * per + (bid >> 3);
}

// Work items of a persistent block. With G blocks and I items, both multiples of 8,
// the blocks dispatched to XCD x (ids congruent to x mod 8) take the items of the
// contiguous range [x*I/8, (x+1)*I/8) in turn, so neighbouring column tiles share
// one L2; otherwise block b takes items b, b + G, ...
struct ItemRange {
    int first, step, end;
};
__device__ __forceinline__ ItemRange xcd_items(int bid, int nblocks, int items) {
    if ((nblocks & 7) == 0 && (items & 7) == 0) {
        const int per = items >> 3, x = bid & 7;
        return ItemRange{x * per + (bid >> 3), nblocks >> 3, (x + 1) * per};
    }
    return ItemRange{bid, nblocks, items};
}


// ---- host helpers -----------------------------------------------------------

#define CWO_DISPATCH_M(M_, ...)              \
    switch (M_) {                             \
        case 16: { constexpr int MM = 16; __VA_ARGS__; } break;     \
        case 32: { constexpr int MM = 32; __VA_ARGS__; } break;     \
        case 64: { constexpr int MM = 64; __VA_ARGS__; } break;     \
        case 128: { constexpr int MM = 128; __VA_ARGS__; } break;   \
        case 256: { constexpr int MM = 256; __VA_ARGS__; } break;   \
        case 512: { constexpr int MM = 512; __VA_ARGS__; } break;   \
        case 1024: { constexpr int MM = 1024; __VA_ARGS__; } break; \
        case 2048: { constexpr int MM = 2048; __VA_ARGS__; } break; \
        case 4096: { constexpr int MM = 4096; __VA_ARGS__; } break; \
        case 8192: { constexpr int MM = 8192; __VA_ARGS__; } break; \
        default: return hipErrorInvalidValue;                 \
    }

// Blocks of a persistent kernel that are resident at once on the current device (at
// most `items`). The occupancy query is answered once per kernel and device.
template <class K>
static int resident_blocks(K kernel, int threads, int items) {
    static std::mutex mu;
    static std::map<std::pair<const void*, int>, long long> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) dev = 0;
    const auto key = std::make_pair(reinterpret_cast<const void*>(kernel), dev);
    long long n = 0;
    {
        std::lock_guard<std::mutex> g(mu);
        auto it = cache.find(key);
        if (it != cache.end()) n = it->second;
    }
    if (n == 0) {
        int cus = 0, occ = 0;
        if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
            cus <= 0)
            cus = 256;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, threads, 0) != hipSuccess ||
            occ <= 0)
            occ = 1;
        n = (long long)occ * cus;
        std::lock_guard<std::mutex> g(mu);
        cache[key] = n;
    }
    return (int)(items < n ? items : n);
}

}  // namespace cwo
