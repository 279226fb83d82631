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

#include <hip/hip_ext.h>

#include "fft_device.hpp"
#include "launch.hpp"

namespace cwo {

// Every kernel of the library is launched through here: a plain launch, or with an armed
// stage timer one whose start and stop events the runtime stamps from the kernel's own
// execution (see StageTimer).
template <class K, class... A>
inline void launch_kernel(K kernel, dim3 grid, dim3 block, size_t shmem, hipStream_t s,
                          A... args) {
    if (StageTimer* t = g_stage_timer) {
        hipExtLaunchKernelGGL(kernel, grid, block, (std::uint32_t)shmem, s,
                              t->started ? nullptr : t->start, t->stop, 0u, args...);
        t->started = true;
    } else {
        hipLaunchKernelGGL(kernel, grid, block, shmem, s, args...);
    }
}

// ---- configuration per transform length --------------------------------------

// Row passes: one transform per thread group of T = M/E threads, RPB rows per block.
template <int M>
struct RowCfg {
    static constexpr int E = 16;
    static constexpr int T = M / E;
    static constexpr int RPB = (T >= 256) ? 1 : 256 / T;  // rows per block
    static constexpr int THREADS = T * RPB;
};

// ---- storage layout of the padded spectrum plane between the passes -------------
//
// Row-major: element (y, x) of the [Ny][Mx] plane at y*Mx + x. Tiled: the columns are
// grouped in tiles of kTileW and each tile stores its rows one after another, element
// (y, x) at ((x / kTileW)*Ny + y)*kTileW + x % kTileW. In the tiled plane the successive
// rows of a column pair lie 8*kTileW bytes apart, so a wavefront of the column pass reads
// and writes a few whole cache lines instead of one line per lane; the row passes move
// whole tile rows of several rows at a time through LDS (RPB rows per block).
constexpr int kTileW = 4;

struct LayRow {
    int mx;
    __device__ __forceinline__ size_t at(int y, int x) const { return (size_t)y * mx + x; }
};
struct LayTile {
    int ny;
    __device__ __forceinline__ size_t at(int y, int x) const {
        return ((size_t)(x / kTileW) * ny + y) * kTileW + (x % kTileW);
    }
};

// Row passes on the tiled plane: RPB rows per block, so that a block moves RPB*kTileW
// contiguous elements per tile (64 bytes of complex64 with two rows); the transform
// results go through LDS once more to be regrouped by tile.
template <int M>
struct TileRowCfg {
    static constexpr int E = 16;
    static constexpr int T = M / E;
    static constexpr int RPB = (T >= 512) ? 1 : (T >= 128 ? 2 : 256 / T);
    static constexpr int THREADS = T * RPB;
    static constexpr int TS = kTileW * RPB;         // LDS float2 per tile
    static constexpr int XCH = RPB * lds_elems<M>();  // exchange buffers of the transforms
    static constexpr int TRN = (M / kTileW) * TS;     // regrouping buffer
    static constexpr int LDS = XCH > TRN ? XCH : TRN;
};

// A row group's tile rows move in 16-byte chunks of CE elements: chunk c of the group sits
// at c*CE in the regrouping buffer (tile t = c / PER_TILE, tile-major) and at
// (t*Ny + y0)*kTileW + (c % PER_TILE)*CE in the plane; CPT chunks per thread.
template <int M, class SE>
struct TileChunks {
    using C = TileRowCfg<M>;
    static constexpr int CE = 16 / (int)sizeof(SE);
    static constexpr int PER_TILE = C::RPB * kTileW / CE;
    static constexpr int CPT = (M / kTileW) * PER_TILE / C::THREADS;
    static_assert(CPT * C::THREADS == (M / kTileW) * PER_TILE, "chunks");
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
