// Host runtime internals shared by the C ABI implementation (capi.hip) and the
// request server (server.hip): the context with its device allocator and the
// HBM pool allocator.  Not part of the public C ABI (include/nlfem.h).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <mutex>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "../../include/nlfem.h"

namespace nlfem {

// One device allocation carved into blocks by best fit, with coalescing of
// neighbouring free blocks.  Thread-safe; every block is 256-byte aligned.
struct Pool {
    std::mutex mu;
    char* base = nullptr;
    size_t size = 0, used = 0, peak = 0;
    std::map<size_t, size_t> by_off;        // free blocks: offset -> bytes
    std::multimap<size_t, size_t> by_size;  // free blocks: bytes -> offset

    bool init(size_t bytes);  // one hipMalloc
    void destroy();           // hipFree of the whole pool
    void* alloc(size_t bytes);  // nullptr when no free block is large enough
    void release(void* p, size_t bytes);
    size_t largest_free();

   private:
    void insert_free(size_t off, size_t bytes);
    void erase_free(std::map<size_t, size_t>::iterator it);
};

}  // namespace nlfem

// Context: device, stream, and the allocator state of everything the library
// holds on the device for the caller.  Without a pool, freed blocks are kept
// in a size-keyed cache for reuse on the same stream (stream order makes the
// reuse safe).  With a pool (server slots), freed blocks are returned to the
// shared pool only after the context's stream has drained, since other
// streams may take them next.
struct nlfem_ctx {
    // guards the allocator state below: the plans of a batch are built by
    // several threads that allocate their plan memory from one context
    std::recursive_mutex mu;
    int device = 0;
    hipStream_t stream = nullptr;
    size_t budget = 0;  // 0 = unlimited
    size_t live = 0, cached = 0, peak = 0;
    std::multimap<size_t, void*> cache;
    std::unordered_map<void*, size_t> sizes;
    nlfem::Pool* pool = nullptr;
    std::vector<std::pair<void*, size_t>> pending;  // pool mode: freed, not yet drained
    std::string err;
    size_t lds_max = 65536;
    double* pinned = nullptr;  // host scratch for readbacks
    int64_t* pinned_i = nullptr;
};

namespace nlfem {

nlfem_status fail(nlfem_ctx* c, nlfem_status s, const std::string& msg);
size_t round_up(size_t b);
void release_cache(nlfem_ctx* c);
// returns nullptr on failure (c->err set)
void* dalloc(nlfem_ctx* c, size_t bytes);
void dfree(nlfem_ctx* c, void* p);
// pool mode: waits for the context's stream, then returns freed blocks to the pool
void drain_pending(nlfem_ctx* c);
// moves the cached (free, idle) blocks of `from` into the cache of `to`; the
// caller has drained from's stream (no pool mode on either side)
void adopt_cache(nlfem_ctx* to, nlfem_ctx* from);

}  // namespace nlfem
