// Device memory management of the library: the per-context caching allocator
// with its HBM budget, and the pool allocator that server slots share.
#include <algorithm>

#include "runtime.hpp"

namespace nlfem {

// ---- pool --------------------------------------------------------------------

bool Pool::init(size_t bytes) {
    bytes &= ~(size_t)255;
    if (bytes == 0) return false;
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return false;
    }
    base = (char*)p;
    size = bytes;
    used = peak = 0;
    by_off.clear();
    by_size.clear();
    insert_free(0, bytes);
    return true;
}

void Pool::destroy() {
    if (base) (void)hipFree(base);
    base = nullptr;
    size = used = 0;
    by_off.clear();
    by_size.clear();
}

void Pool::insert_free(size_t off, size_t bytes) {
    by_off.emplace(off, bytes);
    by_size.emplace(bytes, off);
}

void Pool::erase_free(std::map<size_t, size_t>::iterator it) {
    auto range = by_size.equal_range(it->second);
    for (auto s = range.first; s != range.second; ++s)
        if (s->second == it->first) {
            by_size.erase(s);
            break;
        }
    by_off.erase(it);
}

void* Pool::alloc(size_t bytes) {
    std::lock_guard<std::mutex> g(mu);
    auto it = by_size.lower_bound(bytes);
    if (it == by_size.end()) return nullptr;
    const size_t off = it->second, sz = it->first;
    by_size.erase(it);
    by_off.erase(off);
    if (sz > bytes) insert_free(off + bytes, sz - bytes);
    used += bytes;
    peak = std::max(peak, used);
    return base + off;
}

void Pool::release(void* p, size_t bytes) {
    std::lock_guard<std::mutex> g(mu);
    size_t off = (size_t)((char*)p - base);
    used -= bytes;
    auto next = by_off.find(off + bytes);
    if (next != by_off.end()) {
        bytes += next->second;
        erase_free(next);
    }
    auto prev = by_off.lower_bound(off);
    if (prev != by_off.begin()) {
        --prev;
        if (prev->first + prev->second == off) {
            off = prev->first;
            bytes += prev->second;
            erase_free(prev);
        }
    }
    insert_free(off, bytes);
}

size_t Pool::largest_free() {
    std::lock_guard<std::mutex> g(mu);
    return by_size.empty() ? 0 : by_size.rbegin()->first;
}

// ---- context allocator ---------------------------------------------------------

nlfem_status fail(nlfem_ctx* c, nlfem_status s, const std::string& msg) {
    if (c) c->err = msg;
    return s;
}

size_t round_up(size_t b) { return (b + 255) & ~(size_t)255; }

void release_cache(nlfem_ctx* c) {
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    for (auto& kv : c->cache) (void)hipFree(kv.second);
    c->cache.clear();
    c->cached = 0;
}

void adopt_cache(nlfem_ctx* to, nlfem_ctx* from) {
    std::lock_guard<std::recursive_mutex> lt(to->mu);
    std::lock_guard<std::recursive_mutex> lf(from->mu);
    for (auto& kv : from->cache) to->cache.emplace(kv.first, kv.second);
    to->cached += from->cached;
    from->cache.clear();
    from->cached = 0;
}

void drain_pending(nlfem_ctx* c) {
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    if (!c->pool || c->pending.empty()) return;
    (void)hipStreamSynchronize(c->stream);
    for (auto& b : c->pending) {
        c->pool->release(b.first, b.second);
        c->live -= b.second;
    }
    c->pending.clear();
}

void* dalloc(nlfem_ctx* c, size_t bytes) {
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    bytes = round_up(bytes ? bytes : 1);
    if (c->pool) {
        if (c->budget && c->live + bytes > c->budget) {
            drain_pending(c);
            if (c->live + bytes > c->budget) {
                c->err = "HBM budget exceeded: need " + std::to_string(bytes) + " more bytes, " +
                         std::to_string(c->live) + " in use, budget " + std::to_string(c->budget);
                return nullptr;
            }
        }
        void* p = c->pool->alloc(bytes);
        if (!p) {
            drain_pending(c);
            p = c->pool->alloc(bytes);
        }
        if (!p) {
            c->err = "HBM pool exhausted: need " + std::to_string(bytes) + " bytes, " + std::to_string(c->live) +
                     " held by this slot";
            return nullptr;
        }
        c->live += bytes;
        c->peak = std::max(c->peak, c->live);
        c->sizes[p] = bytes;
        return p;
    }
    auto it = c->cache.lower_bound(bytes);
    if (it != c->cache.end() && it->first <= 2 * bytes) {
        void* p = it->second;
        size_t sz = it->first;
        c->cache.erase(it);
        c->cached -= sz;
        c->live += sz;
        c->peak = std::max(c->peak, c->live);
        c->sizes[p] = sz;
        return p;
    }
    if (c->budget && c->live + c->cached + bytes > c->budget) release_cache(c);
    if (c->budget && c->live + bytes > c->budget) {
        c->err = "HBM budget exceeded: need " + std::to_string(bytes) + " more bytes, " + std::to_string(c->live) +
                 " in use, budget " + std::to_string(c->budget);
        return nullptr;
    }
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        release_cache(c);
        if (hipMalloc(&p, bytes) != hipSuccess) {
            (void)hipGetLastError();
            c->err = "hipMalloc of " + std::to_string(bytes) + " bytes failed";
            return nullptr;
        }
    }
    c->live += bytes;
    c->peak = std::max(c->peak, c->live);
    c->sizes[p] = bytes;
    return p;
}

void dfree(nlfem_ctx* c, void* p) {
    if (!p) return;
    std::lock_guard<std::recursive_mutex> lk(c->mu);
    auto it = c->sizes.find(p);
    if (it == c->sizes.end()) return;
    size_t sz = it->second;
    c->sizes.erase(it);
    if (c->pool) {
        c->pending.emplace_back(p, sz);  // still counted in live until drained
        return;
    }
    c->live -= sz;
    c->cache.emplace(sz, p);
    c->cached += sz;
}

}  // namespace nlfem
