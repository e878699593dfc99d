// Uneven batches: chains of many problems (1 to 6 qubits, any chain count,
// FP64 or the FP32 Kronecker form per problem) in one persistent launch per
// launch class.  The host cuts every problem into workgroup tiles (WG / G_Q
// chains each, G_Q the team size of that qubit count), orders the tiles by
// estimated cost, largest first, and the resident workgroups take tiles from a
// global counter until the list is exhausted.  A tile runs the same chain_tile
// code as a single-problem launch, on its own problem's buffers, so a
// problem's results do not depend on the batch around it.
//
// A launch's register and LDS allocation is that of its largest tile.  The
// 6-qubit tiles need 256 VGPRs and about 150 KB of LDS, which leaves room for
// one 512-thread workgroup per CU (two wavefronts per SIMD); tiles of up to 5
// qubits fit in 128 VGPRs, i.e. twice the resident wavefronts.  So the batch
// runs as up to three launches per precision back to back on the stream: the
// 6-qubit tiles (k_chains_batch<6, .>, 512-thread workgroups), the 5-qubit
// tiles (k_chains_batch<5, .>) and all smaller ones (k_chains_batch<4, .>),
// the last two with 256-thread workgroups.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "chain_kernel.hpp"

namespace qst {

// Launch classes: tiles of 1..4 qubits (class 4), 5-qubit tiles (class 5),
// 6-qubit tiles (class 6).  Workgroup size of each class: 512 threads for
// the 6-qubit tiles (one 512-thread team), 256 otherwise, so that a 5-qubit
// tile is one 256-thread team with barriers of its own, as in its
// single-problem launch.
constexpr int batch_class(int q) { return q <= 4 ? 4 : q; }
constexpr int batch_wg(int qmax) { return qmax == 6 ? 512 : 256; }

struct BatchItem {
    int32_t problem;   // index into the ChainArgs array
    int32_t q;         // qubit count of that problem
    int64_t chain0;    // first chain of the tile
    int32_t prec;      // kPrecF64 or kPrecF32 (the Kronecker forms)
    int32_t pad;
};

struct BatchArgs {
    const ChainArgs* problems;
    const BatchItem* items;
    int32_t n_items;
    int32_t* counter;   // next tile to take; zero at launch
};

// Team size of each qubit count inside a batch launch.
template <int Q>
struct BatchTeam {
    static constexpr int G = Q == 1 ? 8 : Q == 2 ? 16 : Q == 3 ? 32 : Q == 4 ? 64 : Q == 5 ? 256 : 512;
};

template <int Q>
constexpr size_t batch_lds_doubles()
{
    return static_cast<size_t>(batch_wg(batch_class(Q)) / BatchTeam<Q>::G) * TeamShape<Q, BatchTeam<Q>::G>::kLdsChain +
           WgTables<Q>::kDoubles;
}

// One tile of qubit count Q, with the dynamic LDS declared here so that its
// accesses stay LDS instructions when the tile is a callee of its own.
template <int Q, int PREC, int QMAX>
__device__ __forceinline__ void batch_tile_body(const ChainArgs& A, int64_t chain0)
{
    extern __shared__ double batch_lds[];
    static_assert(batch_class(Q) == QMAX, "a tile runs in the launch of its class");
    constexpr int WG = batch_wg(QMAX);
    wg_tables_init<Q>(batch_lds, threadIdx.x, WG);
    __syncthreads();
    chain_tile<Q, BatchTeam<Q>::G, WG, kPathKron, PREC>(A, chain0, batch_lds,
                                                              batch_lds + WgTables<Q>::kDoubles);
}

// In the launch that mixes qubit counts each count is a callee of its own:
// with several chain steps inlined into one body the kernel needed long
// branches and heavy register spilling (and, with all six inlined, its
// 5-qubit tiles computed wrong likelihoods).  The single-count classes inline
// their one tile, as the single-problem kernel does.
template <int Q, int PREC, int QMAX>
__device__ __attribute__((noinline)) void batch_tile(const ChainArgs& A, int64_t chain0)
{
    batch_tile_body<Q, PREC, QMAX>(A, chain0);
}

// The tiles of class QMAX.  The host sorts every tile into the launch of
// its class; a tile of another class is left alone here rather than run with
// the wrong sizes.
template <int PREC, int QMAX>
__device__ __forceinline__ void batch_dispatch(int q, const ChainArgs& A, int64_t chain0)
{
    if constexpr (QMAX == 6) {
        if (q == 6) batch_tile_body<6, PREC, 6>(A, chain0);
    } else if constexpr (QMAX == 5) {
        if (q == 5) batch_tile_body<5, PREC, 5>(A, chain0);
    } else {
        switch (q) {
            case 1: batch_tile<1, PREC, 4>(A, chain0); break;
            case 2: batch_tile<2, PREC, 4>(A, chain0); break;
            case 3: batch_tile<3, PREC, 4>(A, chain0); break;
            case 4: batch_tile<4, PREC, 4>(A, chain0); break;
            default: break;
        }
    }
}

// Wavefronts per SIMD the launch is compiled for: 4 (128 VGPRs) for tiles of
// up to 5 qubits, 2 (256 VGPRs) for 6-qubit tiles.
template <int QMAX>
constexpr int batch_waves_per_simd() { return QMAX == 6 ? 2 : 4; }

// One launch per (class, precision): each holds the tiles of one class in
// one precision, so a single-count class inlines exactly one chain step.
template <int QMAX, int PREC>
__global__ __launch_bounds__(batch_wg(QMAX), batch_waves_per_simd<QMAX>()) void k_chains_batch(BatchArgs B)
{
    __shared__ int32_t take;
    for (;;) {
        if (threadIdx.x == 0) take = atomicAdd(B.counter, 1);
        __syncthreads();
        // the same for every thread: the tile's arguments become scalar loads
        const int32_t it = __builtin_amdgcn_readfirstlane(take);
        __syncthreads();
        if (it >= B.n_items) break;
        const BatchItem I = B.items[it];
        const ChainArgs A = B.problems[I.problem];
        if (I.prec == PREC) batch_dispatch<PREC, QMAX>(I.q, A, I.chain0);
        __syncthreads();
    }
}

__global__ void k_zero_counter(int32_t* c) { c[0] = 0; }

}  // namespace qst
