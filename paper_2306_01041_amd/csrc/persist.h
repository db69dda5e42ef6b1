// Device-side pieces of the persistent (dataflow) sweeps, shared by the
// forward and the reverse sweep: the cache policy of the data that passes
// between wavefronts, the bounded stamp wait and the registration that
// gives work only to running wavefronts. The protocol is described with the
// forward sweep (k_persist.hip).

#pragma once

#include <cstdint>

#include <hip/hip_runtime.h>

namespace vrt_persist {

// Scope of the polls and stamps: relaxed agent-scope atomics (sc1)
constexpr int kXScope = __HIP_MEMORY_SCOPE_AGENT;
// cache-policy bits of the intensity-row buffer accesses: sc1 (device scope)
constexpr int kRowPolicy = 16;
// buffer descriptor word 3 of an untyped 32-bit buffer on gfx9 targets
constexpr int kRawBufferWord3 = 0x00020000;

// Device-scope loads and stores of 4, 8 or 16 bytes at byte offset `off` of
// the buffer `r` (one ray's block of intensity rows)
template <typename X> __device__ __forceinline__ X row_load(__amdgpu_buffer_rsrc_t r, uint32_t off) {
  if constexpr (sizeof(X) == 16) {
    return __builtin_bit_cast(X, __builtin_amdgcn_raw_buffer_load_b128(r, off, 0, kRowPolicy));
  } else if constexpr (sizeof(X) == 8) {
    return __builtin_bit_cast(X, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, kRowPolicy));
  } else {
    return __builtin_bit_cast(X, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, kRowPolicy));
  }
}
template <typename X> __device__ __forceinline__ void row_store(__amdgpu_buffer_rsrc_t r, uint32_t off, const X &v) {
  if constexpr (sizeof(X) == 16) {
    typedef uint32_t U __attribute__((ext_vector_type(4)));
    __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(U, v), r, off, 0, kRowPolicy);
  } else if constexpr (sizeof(X) == 8) {
    typedef uint32_t U __attribute__((ext_vector_type(2)));
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(U, v), r, off, 0, kRowPolicy);
  } else {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, off, 0, kRowPolicy);
  }
}

// One ray's block of rows accessed with the device-scope policy, at byte
// offsets. Below 4 GiB one descriptor covers the whole block, uniform across
// the wavefront. Above (BIG), every access takes the descriptor of the 2 GiB
// window holding its offset; the descriptor then differs between lanes, and
// the compiler issues the access once per distinct window in the wavefront.
template <bool BIG> struct RayBlock {
  __amdgpu_buffer_rsrc_t whole;
  char *base;
  int64_t bytes;
  __device__ __forceinline__ RayBlock(const void *p, int64_t nbytes)
      : base(static_cast<char *>(const_cast<void *>(p))), bytes(nbytes) {
    if constexpr (!BIG) whole = __builtin_amdgcn_make_buffer_rsrc(base, 0, (int)(uint32_t)nbytes, kRawBufferWord3);
  }
  __device__ __forceinline__ __amdgpu_buffer_rsrc_t window(int64_t w) const {
    const int64_t rest = bytes - (w << 31);
    const int64_t lim = rest < 0xffffffffLL ? rest : 0xffffffffLL;
    return __builtin_amdgcn_make_buffer_rsrc(base + (w << 31), 0, (int)(uint32_t)lim, kRawBufferWord3);
  }
  template <typename X> __device__ __forceinline__ X load(int64_t off) const {
    if constexpr (BIG) {
      const int64_t w = off >> 31;
      return row_load<X>(window(w), (uint32_t)(off - (w << 31)));
    } else {
      return row_load<X>(whole, (uint32_t)off);
    }
  }
  template <typename X> __device__ __forceinline__ void store(int64_t off, const X &v) const {
    if constexpr (BIG) {
      const int64_t w = off >> 31;
      row_store<X>(window(w), (uint32_t)(off - (w << 31)), v);
    } else {
      row_store<X>(whole, (uint32_t)off, v);
    }
  }
};

constexpr int32_t kFrozen = 1 << 30;

// Wait until *f == epoch. Returns false if the bound was exceeded or another
// wave already gave up (then the caller proceeds without the data).
__device__ __forceinline__ bool wait_stamp(const int32_t *f, int32_t epoch, int32_t *err, int64_t cap) {
  int64_t it = 0;
  while (__hip_atomic_load(f, __ATOMIC_RELAXED, kXScope) != epoch) {
    ++it;
    if ((it & 63) == 0 && __hip_atomic_load(err, __ATOMIC_RELAXED, kXScope) != 0) return false;
    if (it > cap) {
      __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, kXScope);
      return false;
    }
    __builtin_amdgcn_s_sleep(1);
  }
  return true;
}

// polls without a new registration after which the count is frozen
constexpr int32_t kStallPolls = 512;

// Registration (wave-uniform): returns this wavefront's rank and sets W, or
// returns -1 for a wavefront that registered after the freeze. The first
// wavefront polls until `total` have registered, the count has not changed
// for kStallPolls polls, or `cap` polls have passed.
__device__ __forceinline__ int64_t register_wave(int32_t *words, int32_t total, int64_t cap, int lane,
                                                 int64_t &W) {
  int32_t *reg = words + 2, *frozen = words + 3, *err = words + 1;
  int32_t old = 0;
  if (lane == 0) old = __hip_atomic_fetch_add(reg, 1, __ATOMIC_RELAXED, kXScope);
  old = __builtin_amdgcn_readfirstlane(old);
  if (old & kFrozen) return -1;
  if (old == 0) {
    int64_t it = 0;
    int32_t last = -1, still = 0;
    for (;;) {
      const int32_t c = __hip_atomic_load(reg, __ATOMIC_RELAXED, kXScope);
      if (c >= total || ++it > cap) break;
      if (c == last) {
        if (++still > kStallPolls) break;
      } else {
        last = c;
        still = 0;
      }
      __builtin_amdgcn_s_sleep(8);
    }
    int32_t got = 0;
    if (lane == 0) {
      got = __hip_atomic_fetch_or(reg, kFrozen, __ATOMIC_RELAXED, kXScope) & (kFrozen - 1);
      __hip_atomic_store(frozen, got + 1, __ATOMIC_RELAXED, kXScope);
    }
    W = __builtin_amdgcn_readfirstlane(got);
    return 0;
  }
  int64_t it = 0;
  int32_t f;
  while ((f = __hip_atomic_load(frozen, __ATOMIC_RELAXED, kXScope)) == 0) {
    if (++it > cap) {
      __hip_atomic_fetch_or(err, 1, __ATOMIC_RELAXED, kXScope);
      return -1;
    }
    __builtin_amdgcn_s_sleep(8);
  }
  W = __builtin_amdgcn_readfirstlane(f - 1);
  return old;
}

}  // namespace vrt_persist
