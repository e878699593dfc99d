// Uneven batches: chains of many problems (1 to 6 qubits, any chain count,
// FP64 or the FP32 Kronecker form per problem) in one launch per launch
// class.  The host cuts every problem into workgroup tiles (WG / G_Q chains
// each, G_Q the team size of that qubit count) and orders the tiles by
// estimated cost, largest first; in a persistent launch the resident
// workgroups take tiles from a global counter until the list is exhausted,
// and the 6-qubit class runs as a plain grid of one workgroup per tile in that
// order.  A tile runs the same chain_tile code as a single-problem launch, on
// its own problem's buffers, so a problem's results do not depend on the
// batch around it.
//
// A launch's register and LDS allocation is that of its largest tile.  A
// 6-qubit tile needs about 150 KB of LDS, which leaves room for one
// workgroup per CU: its 1024-thread team fills it (four wavefronts per SIMD
// at 128 VGPRs), while the smaller tiles would lose most of their resident
// workgroups in such a launch.  So the batch runs as one launch per qubit
// count and precision present: k_chains_batch<Q, precision> with 256-thread
// workgroups up to 5 qubits, k_chains_batch_grid<6, precision> with 1024.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "chain_kernel.hpp"

namespace qst {

// Launch classes: one per qubit count.  Workgroup size of each class: 1024
// threads for the 6-qubit tiles (one 1024-thread team), 256 otherwise, so
// that a 5-qubit tile is one 256-thread team with barriers of its own, as in
// its single-problem launch.
constexpr int batch_class(int q) { return q; }
constexpr int batch_wg(int qmax) { return qmax == 6 ? 1024 : 256; }

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
    static constexpr int G = Q == 1 ? 8 : Q == 2 ? 16 : Q == 3 ? 32 : Q == 4 ? 64 : Q == 5 ? 256 : 1024;
};

template <int Q>
constexpr size_t batch_lds_doubles()
{
    return static_cast<size_t>(batch_wg(batch_class(Q)) / BatchTeam<Q>::G) * TeamShape<Q, BatchTeam<Q>::G>::kLdsChain +
           WgTables<Q>::kDoubles;
}

// What a tile touches fits what its launch is given: chain_tile addresses
// the workgroup tables [0, WgTables::kDoubles) and WG / G team regions of
// kLdsChain doubles after them, and the host passes batch_lds_doubles<Q>()
// for the class of Q; the workgroup holds whole teams, and the total stays
// within the 160 KB of LDS of a gfx950 CU.
template <int Q>
constexpr bool batch_layout_ok()
{
    constexpr int WG = batch_wg(batch_class(Q)), G = BatchTeam<Q>::G;
    return WG % G == 0 && batch_lds_doubles<Q>() * sizeof(double) <= 160 * 1024 &&
           batch_lds_doubles<Q>() ==
               WgTables<Q>::kDoubles + static_cast<size_t>(WG / G) * TeamShape<Q, G>::kLdsChain;
}
static_assert(batch_layout_ok<1>() && batch_layout_ok<2>() && batch_layout_ok<3>() && batch_layout_ok<4>() &&
                  batch_layout_ok<5>() && batch_layout_ok<6>(),
              "batch tile LDS layout");

// One tile of qubit count Q, inlined into the launch of its class as the
// single-problem kernel inlines its chain step.  (One launch for all qubit
// counts, with each count's tile as a callee of its own, needed long
// branches and heavy register spilling; with all six inlined into one body
// its 5-qubit tiles computed wrong likelihoods.)
template <int Q, int PREC>
__device__ __forceinline__ void batch_tile(const ChainArgs& A, int64_t chain0)
{
    extern __shared__ double batch_lds[];
    constexpr int WG = batch_wg(Q);
    wg_tables_init<Q>(batch_lds, threadIdx.x, WG);
    __syncthreads();
    chain_tile<Q, BatchTeam<Q>::G, WG, kPathKron, PREC>(A, chain0, batch_lds,
                                                              batch_lds + WgTables<Q>::kDoubles);
}

// Wavefronts per SIMD the launch is compiled for: 4 (128 VGPRs) for every
// class (a 6-qubit workgroup alone brings four).
template <int QMAX>
constexpr int batch_waves_per_simd() { return 4; }

// One launch per (qubit count, precision), inlining exactly one chain step.
// The host sorts every tile into the launch of its class; a tile of another
// class is left alone here rather than run with the wrong sizes.
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
        if (I.q == QMAX && I.prec == PREC) batch_tile<QMAX, PREC>(A, I.chain0);
        __syncthreads();
    }
}

// The 6-qubit class as a plain grid, one workgroup per tile in the list's
// largest-first order: with one workgroup per CU and tiles of milliseconds,
// the work queue gains nothing there, and its loop around the tile cost the
// tile's registers (340 and 300 bytes of spills per lane in FP64 and FP32,
// 180 and 148 without it, against 172 and 140 in the single-problem kernel).
template <int QMAX, int PREC>
__global__ __launch_bounds__(batch_wg(QMAX), batch_waves_per_simd<QMAX>()) void k_chains_batch_grid(BatchArgs B)
{
    const BatchItem I = B.items[blockIdx.x];
    const ChainArgs A = B.problems[I.problem];
    if (I.q == QMAX && I.prec == PREC) batch_tile<QMAX, PREC>(A, I.chain0);
}

__global__ void k_zero_counter(int32_t* c) { c[0] = 0; }

__global__ void k_zero_counters(int32_t* c, int n)
{
    for (int i = threadIdx.x; i < n; i += blockDim.x) c[i] = 0;
}

}  // namespace qst
