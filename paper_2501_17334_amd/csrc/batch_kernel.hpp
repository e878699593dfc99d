// Uneven batches: chains of many problems (1 to 6 qubits, any chain count,
// FP64 or the FP32 Kronecker form per problem) in ONE persistent launch.  The host cuts every problem into workgroup
// tiles (WG / G_Q chains each, G_Q the team size of that qubit count), orders
// the tiles by estimated cost, largest first, and the resident workgroups
// take tiles from a global counter until the list is exhausted.  A tile runs
// the same chain_tile code as a single-problem launch, on its own problem's
// buffers, so a problem's results do not depend on the batch around it.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "chain_kernel.hpp"

namespace qst {

constexpr int kBatchWG = 512;

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
    return static_cast<size_t>(kBatchWG / BatchTeam<Q>::G) * TeamShape<Q, BatchTeam<Q>::G>::kLdsChain +
           WgTables<Q>::kDoubles;
}

// One tile of qubit count Q.  Each qubit count is a callee of its own, with
// the dynamic LDS declared here so that its accesses stay LDS instructions:
// with all six chain steps inlined into one body the kernel needed long
// branches and heavy register spilling, and its 5-qubit tiles computed wrong
// likelihoods.
template <int Q, int PREC>
__device__ __attribute__((noinline)) void batch_tile(const ChainArgs& A, int64_t chain0)
{
    extern __shared__ double batch_lds[];
    wg_tables_init<Q>(batch_lds, threadIdx.x, kBatchWG);
    __syncthreads();
    chain_tile<Q, BatchTeam<Q>::G, kBatchWG, kPathKron, PREC>(A, chain0, batch_lds,
                                                              batch_lds + WgTables<Q>::kDoubles);
}

template <int PREC>
__device__ __forceinline__ void batch_dispatch(int q, const ChainArgs& A, int64_t chain0)
{
    switch (q) {
        case 1: batch_tile<1, PREC>(A, chain0); break;
        case 2: batch_tile<2, PREC>(A, chain0); break;
        case 3: batch_tile<3, PREC>(A, chain0); break;
        case 4: batch_tile<4, PREC>(A, chain0); break;
        case 5: batch_tile<5, PREC>(A, chain0); break;
        default: batch_tile<6, PREC>(A, chain0); break;
    }
}

__global__ __launch_bounds__(kBatchWG, 2) void k_chains_batch(BatchArgs B)
{
    __shared__ int32_t take;
    for (;;) {
        if (threadIdx.x == 0) take = atomicAdd(B.counter, 1);
        __syncthreads();
        const int32_t it = take;
        __syncthreads();
        if (it >= B.n_items) break;
        const BatchItem I = B.items[it];
        const ChainArgs A = B.problems[I.problem];
        if (I.prec == kPrecF32) batch_dispatch<kPrecF32>(I.q, A, I.chain0);
        else batch_dispatch<kPrecF64>(I.q, A, I.chain0);
        __syncthreads();
    }
}

__global__ void k_zero_counter(int32_t* c) { c[0] = 0; }

}  // namespace qst
