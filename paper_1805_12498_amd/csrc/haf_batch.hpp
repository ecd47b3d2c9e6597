// Work description of the persistent batched kernel, shared by the host planner
// (batched calls and the request server) and the kernel.
//
// A launch runs a list of classes.  A class is the subsets of one size m of one
// item (all with s = 2m rows and sign (-1)^(N-m)), cut into chunks of `cap`
// consecutive ranks; chunk j of a class covers ranks [j cap, min((j+1) cap, total)).
// The classes of a launch are ordered by decreasing cost per chunk and numbered
// through by chunk_base, so that a global chunk counter hands the largest chunks
// out first.  Every chunk leaves one double-double partial in a slot that depends
// only on the item (slot0 + slot_base + j); the wave that completes an item's
// last chunk folds the item's slots in slot order.  Hence an item's result does
// not depend on what else is in the launch, nor on which wave ran which chunk.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hafgpu {

constexpr int kBatchMaxS = 48;        // largest subset the batched kernel has a layout for
constexpr int kBatchMaxCap = 64;      // subsets per chunk (one series lane each)

enum BatchItemKind : int {
    kItemComputed = -1,               // computed by the batched kernel
    kItemZero = 0,                    // constant result 0 (haf of odd n)
    kItemOne = 1,                     // constant result 1 (n = 0)
    kItemExternal = 2,                // handled outside the batched kernel (n > kBatchMaxS)
};

struct BatchItem {
    const double2* A;                 // matrix read by the kernel (dense copy for odd-n loop hafnians)
    const double2* src;               // caller's matrix; the prologue pads it into A when they differ
    double2* out;                     // result, or null
    double* out_dd;                   // double-double result (re_hi, re_lo, im_hi, im_lo), or null
    int64_t slot0;                    // first partial slot of the item
    int n, lda;                       // matrix read by the kernel: n even
    int src_n, src_lda;
    int loops;                        // 1 = loop hafnian
    int nslots;                       // chunks of the item over all launches = its partial slots
    int kind;                         // BatchItemKind
    int pad_;
};

struct BatchClass {
    int item, m;
    int cap;                          // subsets per chunk
    int total;                        // subsets in the class, C(N, m)
    int j0;                           // first chunk of the class in this launch
    int chunk_base;                   // launch-wide number of that chunk (ascending over classes)
    int slot_base;                    // item-relative slot of chunk 0 of the class
    int pad_;
};

}  // namespace hafgpu
