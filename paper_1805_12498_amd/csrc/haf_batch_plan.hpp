// Host planner of the persistent batched kernel, shared by batched calls and the
// request server.
#pragma once
#include <stdint.h>

#include <vector>

#include "haf_batch.hpp"
#include "hafgpu.h"

namespace hafgpu {

struct ItemShape {
    int kind;         // BatchItemKind
    int n;            // matrix the kernel reads (odd-n loop hafnians padded to n + 1)
    int N;            // n / 2
    bool loops;
    bool padded;
};

// How a matrix of n_src rows and the given kind is computed.
ItemShape classify_item(int n_src, int kind);

haf_batched_config batch_config();

// Layout table for s-row subsets under the configured layout (table 2 above
// s = 32) and the kernel variant that runs the chunks of s <= 32 when the
// largest item has n = 2 max_N.
int cap_table(int layout, int s);
int small_variant(int layout, int max_N);
constexpr int kBigVariant = 2;

// Subsets per chunk for s-row subsets: the matrix slots of a wave (W of them)
// each take group_work (16/s)^3 subsets, at least one, at most 64 per wave.
// A function of (layout, s, group_work) only, so the cut of a matrix does not
// depend on what else shares the launch.
int chunk_cap(int layout, int s, int group_work);

// Appends the classes of one item (m = 1..N, j0 = 0, item-relative slot bases)
// and returns the item's number of chunks = partial slots.
int item_classes(int layout, int group_work, int item, int N, std::vector<BatchClass>* out);

// Orders the classes of a launch by decreasing cost per chunk (ties: item,
// then m) and numbers their chunks; njobs[c] is the number of chunks class c
// runs in this launch.  Returns the launch's chunk count.
int64_t order_classes(int layout, std::vector<BatchClass>& cls, std::vector<int>& njobs);

// Model flops of the subsets of nchunks_here chunks of a class from chunk j0 on.
double class_model_flops(const BatchClass& c, int N, bool loops, int nchunks_here);

// A whole batch: launch 0 takes the chunks with s > 32 (kernel variant 2),
// launch 1 those with s <= 32 (the configured variant); each has its own chunk
// counter, and an item's completion count spans both.
struct BatchPlan {
    std::vector<ItemShape> shapes;
    std::vector<int> item_slots;
    std::vector<int64_t> slot0;
    int64_t nslots = 0;
    int64_t pad_elems = 0;
    std::vector<BatchClass> cls[2];
    std::vector<int> njobs[2];
    int64_t nchunks[2] = { 0, 0 };
    int variant[2] = { kBigVariant, 0 };
    double flops[2] = { 0.0, 0.0 };
};
int plan_batch(const int32_t* ns, const uint8_t* kinds, int count, const haf_batched_config& cfg, BatchPlan* p);

}  // namespace hafgpu
