// Global-memory access helpers: plain or non-temporal (streaming) loads/stores.
#pragma once

#include "common.h"

namespace qs {

template <bool NT, typename V> __device__ __forceinline__ V ld(const V *p) {
    if constexpr (NT)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

template <bool NT, typename V> __device__ __forceinline__ void st(V *p, V v) {
    if constexpr (NT)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

template <typename V> __device__ __forceinline__ void st_nt(V *p, V v) { __builtin_nontemporal_store(v, p); }

}  // namespace qs
