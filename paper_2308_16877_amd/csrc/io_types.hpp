// Element types of the region's columns: the kernels compute in registers
// (float for the region interface) and convert when a column is loaded or
// stored.  BF16 is handled as raw 16-bit patterns.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hpac {

__device__ __forceinline__ float bf16_bits_to_float(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// Round to nearest, ties to even (NaN kept quiet): gfx950's conversion
// instruction (v_cvt_pk_bf16_f32).
__device__ __forceinline__ uint16_t float_to_bf16_bits(float f) { return __builtin_bit_cast(uint16_t, (__bf16)f); }

struct IoF32 {
  using elem = float;
  __device__ __forceinline__ static float load(const void *p, int64_t i) { return ((const float *)p)[i]; }
  __device__ __forceinline__ static void store(void *p, int64_t i, float v) { ((float *)p)[i] = v; }
};
struct IoF16 {
  using elem = _Float16;
  __device__ __forceinline__ static float load(const void *p, int64_t i) { return (float)((const _Float16 *)p)[i]; }
  __device__ __forceinline__ static void store(void *p, int64_t i, float v) { ((_Float16 *)p)[i] = (_Float16)v; }
};
struct IoBF16 {
  using elem = uint16_t;
  __device__ __forceinline__ static float load(const void *p, int64_t i) {
    return bf16_bits_to_float(((const uint16_t *)p)[i]);
  }
  __device__ __forceinline__ static void store(void *p, int64_t i, float v) {
    ((uint16_t *)p)[i] = float_to_bf16_bits(v);
  }
};

// A region evaluated as Base with columns of element type Io.
template <class Base, class Io>
struct WithIo : Base {
  using io = Io;
};

// The same columns read and written with nontemporal (streaming) accesses.
// A grid-stride loop over several items per lane keeps many widely spaced
// streams in flight (each lane's consecutive items lie L apart), and there
// streaming accesses measured faster; a launch of one item per lane, one
// contiguous sweep, measured slower with them, so it keeps ordinary ones.
template <class Io>
struct StreamIo {
  using elem = typename Io::elem;
  __device__ __forceinline__ static float load(const void *p, int64_t i) {
    const elem e = __builtin_nontemporal_load(&((const elem *)p)[i]);
    return Io::load(&e, 0);
  }
  __device__ __forceinline__ static void store(void *p, int64_t i, float v) {
    elem e;
    Io::store(&e, 0, v);
    __builtin_nontemporal_store(e, &((elem *)p)[i]);
  }
};

template <class Base>
struct Streamed : Base {
  using io = StreamIo<typename Base::io>;
};

}  // namespace hpac
