// MFMA geometry, LDS streaming and the activations shared by the forward
// (tmlp_kernels.h) and the adjoint (adjoint_kernels.h) T-MLP kernels on gfx950.
#pragma once

#include "sand_internal.h"

#ifndef SAND_PD
#define SAND_PD 1
#endif
#ifndef SAND_FWD_WAVES
#define SAND_FWD_WAVES 8
#endif

namespace sand {
namespace mfma {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Per-precision MFMA geometry. For lane l: `col` is its point within the
// wavefront's block, `grp` its row group; accumulator register e holds one
// unit of the current output block (see tail_row and put).
template <int PREC>
struct Tr;

template <>
struct Tr<PREC_FP32> {
  using V = float;
  using Acc = f32x4;
  static constexpr int BM = 16;   // units per output block
  static constexpr int NQ = 16;   // points per wavefront
  static constexpr int NR = 4;    // accumulator registers per lane
  static constexpr int SPB = 4;   // K steps per block of input units
  static constexpr int VB = 4;    // A-operand bytes per lane per K step
  static constexpr int L1S = 1;   // layer-1 MFMA steps
  // layer 1: FP32 MFMA, K = (x, y, z, 1); A-operand bytes per step
  using L1V = float;
  static constexpr int L1AB = 256;
  __device__ __forceinline__ static int col(int lane) { return lane & 15; }
  __device__ __forceinline__ static int grp(int lane) { return lane >> 4; }
  __device__ __forceinline__ static Acc mma(V a, V b, Acc c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static Acc mma1(float a, float b, Acc c) { return mma(a, b, c); }
  __device__ __forceinline__ static float l1_a(const char* ch, int step, int lane) {
    return ((const float*)ch)[step * 64 + lane];
  }
  __device__ __forceinline__ static float l1_b(int step, int g, float x, float y, float z) {
    return g == 0 ? x : g == 1 ? y : g == 2 ? z : 1.0f;
  }
  __device__ __forceinline__ static V bias_b(int g) { return g == 0 ? 1.0f : 0.0f; }
  // offset (in floats) of the 4 tail rows that registers 4i..4i+3 hold
  __device__ __forceinline__ static int tail_row(int i, int g) { return 4 * g; }
  // forward-chunk tail weights: a0[BM], a1[BM] in unit order
  static constexpr int TAILB = BM * 8;
  __device__ __forceinline__ static f32x4 tail_vec(const char* tails, int f, int i, int g) {
    return *(const f32x4*)(tails + (f * BM + tail_row(i, g)) * 4);
  }
  template <int KS>
  __device__ __forceinline__ static void put(V (&act)[KS], int rb, int e, float v) {
    act[4 * rb + e] = v;
  }
  // store a block's NR values (in register order) as next-layer B operands
  template <int KS>
  __device__ __forceinline__ static void store(V (&act)[KS], int rb, const float (&h)[NR]) {
#pragma unroll
    for (int e = 0; e < NR; ++e) act[4 * rb + e] = h[e];
  }
  __device__ __forceinline__ static float lane_sum(float v) {
    v += __shfl_xor(v, 16);
    return v + __shfl_xor(v, 32);
  }
};

// v = h + m + l exactly, each part a BF16 (round to nearest even): the
// residuals v - h and v - h - m are exact in FP32, and after two 8-bit parts
// at most 8 significant bits remain.
__device__ __forceinline__ void split3_bf16(float v, __bf16& h, __bf16& m, __bf16& l) {
  h = (__bf16)v;
  const float r = v - (float)h;
  m = (__bf16)r;
  l = (__bf16)(r - (float)m);
}

template <int PREC>
struct Tr16 {
  using Acc = f32x16;
  // Layer 1 of the 16-bit paths runs on BF16 MFMAs with the weights (host)
  // and the coordinates split three ways, w = wh + wm + wl and c = ch + cm +
  // cl: the six partial products of order 2^-16 and above (wh ch, wh cm,
  // wm ch, wh cl, wm cm, wl ch), exact in BF16 x BF16 and summed in FP32,
  // give the omega-scaled argument to about 2^-24 relative, as an FP32
  // product would. K slots (step, lane half): (0, 0) the six products of x
  // and the bias parts bh, bm; (0, 1) those of y and bl; (1, 0) those of z;
  // (1, 1) zero. An FP32 MFMA would hold the vector ALU for its whole
  // duration; the BF16 ones run beside the sines.
  using L1V = bf16x8;
  static constexpr int L1AB = 64 * 16;
  __device__ __forceinline__ static Acc mma1(bf16x8 a, bf16x8 b, Acc c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static bf16x8 l1_a(const char* ch, int step, int lane) {
    return *(const bf16x8*)(ch + (step * 64 + lane) * 16);
  }
  __device__ __forceinline__ static bf16x8 l1_b(int step, int g, float x, float y, float z) {
    const float c = step == 0 ? (g == 0 ? x : y) : (g == 0 ? z : 0.0f);
    __bf16 h, m, l;
    split3_bf16(c, h, m, l);
    const __bf16 one = (__bf16)(step == 0 ? 1.0f : 0.0f);
    const __bf16 one0 = (__bf16)(step == 0 && g == 0 ? 1.0f : 0.0f);
    return bf16x8{h, m, h, l, m, h, one, one0};
  }
  // store a block's NR values (in register order) as next-layer B operands,
  // each 8-wide vector built fresh so no earlier contents stay live
  template <class V, class E, int KS>
  __device__ __forceinline__ static void store16(V (&act)[KS], int rb, const float (&h)[16]) {
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      V v;
#pragma unroll
      for (int p = 0; p < 8; ++p) v[p] = (E)h[8 * q + p];
      act[2 * rb + q] = v;
    }
  }
  static constexpr int BM = 32;
  static constexpr int NQ = 32;
  static constexpr int NR = 16;
  static constexpr int SPB = 2;
  static constexpr int VB = 16;
  static constexpr int L1S = 2;
  __device__ __forceinline__ static int col(int lane) { return lane & 31; }
  __device__ __forceinline__ static int grp(int lane) { return lane >> 5; }
  __device__ __forceinline__ static int tail_row(int i, int g) { return 8 * i + 4 * g; }
  // forward-chunk tail weights, lane-indexed: for factor f, lane l holds the
  // weight of the unit in its own register e = l & 15 (row group g = l >> 5),
  // i.e. a_f[tail_row(e / 4, g) + e % 4]; a DPP row broadcast of lane e then
  // hands every lane of a 16-lane row the weight of its register e.
  static constexpr int TAILB = 2 * 64 * 4;
  __device__ __forceinline__ static f32x4 tail_vec(const char* tails, int f, int i, int g) {
    return *(const f32x4*)(tails + (f * 64 + 32 * g + 4 * i) * 4);
  }
  __device__ __forceinline__ static float lane_sum(float v) { return v + __shfl_xor(v, 32); }
};

template <>
struct Tr<PREC_BF16> : Tr16<PREC_BF16> {
  using V = bf16x8;
  using E = __bf16;
  __device__ __forceinline__ static Acc mma(V a, V b, Acc c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static V bias_b(int g) {
    const __bf16 one = (__bf16)(g == 0 ? 1.0f : 0.0f), z = (__bf16)0.0f;
    return V{one, one, z, z, z, z, z, z};
  }
  template <int KS>
  __device__ __forceinline__ static void put(V (&act)[KS], int rb, int e, float v) {
    act[2 * rb + (e >> 3)][e & 7] = (__bf16)v;
  }
  template <int KS>
  __device__ __forceinline__ static void store(V (&act)[KS], int rb, const float (&h)[16]) {
    store16<V, E, KS>(act, rb, h);
  }
};

template <>
struct Tr<PREC_FP16> : Tr16<PREC_FP16> {
  using V = f16x8;
  using E = _Float16;
  __device__ __forceinline__ static Acc mma(V a, V b, Acc c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_f16(a, b, c, 0, 0, 0);
  }
  __device__ __forceinline__ static V bias_b(int g) {
    const _Float16 one = (_Float16)(g == 0 ? 1.0f : 0.0f), z = (_Float16)0.0f;
    return V{one, one, z, z, z, z, z, z};
  }
  template <int KS>
  __device__ __forceinline__ static void put(V (&act)[KS], int rb, int e, float v) {
    act[2 * rb + (e >> 3)][e & 7] = (_Float16)v;
  }
  template <int KS>
  __device__ __forceinline__ static void store(V (&act)[KS], int rb, const float (&h)[16]) {
    store16<V, E, KS>(act, rb, h);
  }
};

__device__ __forceinline__ float sin_rev(float x) { return __builtin_amdgcn_sinf(x); }

// Argument, in revolutions, of a hidden unit's sine. The accumulator holds
// u = omega z / (2 pi) (the packed weights carry omega / (2 pi)). SIREN's
// sin(omega z) takes u itself; FINER's sin(omega (|z| + 1) z) takes
// u (1 + |z|), with |z| = |u| kf and kf = 2 pi / omega.
template <int ACT>
__device__ __forceinline__ float act_arg(float u, float kf) {
  if constexpr (ACT == ACT_FINER)
    return u * fmaf(fabsf(u), kf, 1.0f);
  else
    return u;
}

// The activation's slope divided by omega, at accumulator value u with
// argument arg = act_arg(u, kf): cos(omega z) for SIREN, and for FINER
// (2|z| + 1) cos(omega (|z| + 1) z) (d/dz of (|z| + 1) z is 2|z| + 1).
template <int ACT>
__device__ __forceinline__ float act_slope(float u, float arg, float kf) {
  if constexpr (ACT == ACT_FINER)
    return __builtin_amdgcn_cosf(arg) * fmaf(fabsf(u), 2.0f * kf, 1.0f);
  else
    return __builtin_amdgcn_cosf(arg);
}

template <int PREC, int WP>
struct Cfg {
  using T = Tr<PREC>;
  static constexpr int NW = 8;                  // adjoint: wavefronts per workgroup
  static constexpr int NT = NW * 64;
  // forward: NWF wavefronts per workgroup, WGF workgroups per CU (two
  // wavefronts per SIMD either way)
  // (layers wider than 256 keep one workgroup of eight: two rings would not
  // fit in the CU's LDS)
  static constexpr int NWF = WP > 256 ? 8 : SAND_FWD_WAVES;
  static constexpr int NTF = NWF * 64;
  static constexpr int WGF = 8 / NWF;
  static constexpr int QF = NWF * T::NQ;         // forward points per tile
  static constexpr int Q = NW * T::NQ;          // points per tile
  static constexpr int RB = WP / T::BM;         // output blocks per layer
  static constexpr int KS = RB * T::SPB;        // K steps of a hidden product
  // compacted dynamic exit: a point's record is a 16-byte header (index, y)
  // and the packed layer output held by its GL lanes, KS vectors each
  static constexpr int GL = 64 / T::NQ;
  static constexpr int REC = 16 + GL * KS * T::VB;
  // forward chunk: KS weight steps + 1 bias step, then tail weights
  static constexpr int TAIL_OFF = (KS + 1) * 64 * T::VB;
  static constexpr int CH = TAIL_OFF + T::TAILB;
  // adjoint chunk (transposed weights, no bias), then tail weights
  static constexpr int TAIL_OFF_B = KS * 64 * T::VB;
  static constexpr int CH_B = TAIL_OFF_B + T::BM * 8;
  static constexpr int L1C = T::L1S * T::L1AB + T::TAILB;    // layer-1 chunk bytes
  static constexpr int L1B = RB * L1C;
  static constexpr int PD = SAND_PD;                     // forward chunks in flight
  static constexpr int NSLOT = PD + 2;                   // forward LDS ring slots
  static constexpr int LDS = NSLOT * CH + L1B;
  static_assert(CH % 16 == 0 && CH_B % 16 == 0 && L1B % 16 == 0,
                "chunks are whole 16-byte pieces");
};

typedef __attribute__((address_space(3))) void lds_void;

// LDS pointer of a generic pointer into a __shared__ array: the low 32 bits
// of a flat address in the LDS aperture are the LDS offset. (A plain cast
// inserts a null check that the gfx950 backend can fail to select.)
#pragma clang diagnostic push
#pragma clang diagnostic ignored "-Wint-to-void-pointer-cast"
__device__ __forceinline__ lds_void* lds_ptr(const void* p) {
  return (lds_void*)(uint32_t)(uintptr_t)p;
}
#pragma clang diagnostic pop

// Start copying one chunk of BYTES bytes from global memory into an LDS slot
// without passing through registers: each wavefront-wide load moves 64
// pieces of 16 bytes to 1 KB of LDS. Completion is awaited (vmcnt) before the
// next workgroup barrier.
template <int BYTES, int NW>
__device__ __forceinline__ void load_chunk(const char* __restrict__ src, char* dst, int wave,
                                           int lane) {
  constexpr int NP = BYTES / 16;
  constexpr int WL = (NP + 64 * NW - 1) / (64 * NW);
#pragma unroll
  for (int k = 0; k < WL; ++k) {
    const int q = k * NW + wave;
    const int piece = q * 64 + lane;
    if (q * 64 < NP && piece < NP)
      __builtin_amdgcn_global_load_lds((const void*)(src + piece * 16), lds_ptr(dst + q * 1024), 16,
                                       0, 0);
  }
}

__device__ __forceinline__ void wait_chunk() { asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); }

// Number of loads one wavefront issues in load_chunk<BYTES, NW>.
template <int BYTES, int NW>
__device__ __forceinline__ int chunk_loads(int wave) {
  constexpr int NP = BYTES / 16;
  constexpr int WL = (NP + 64 * NW - 1) / (64 * NW);
  int n = 0;
#pragma unroll
  for (int k = 0; k < WL; ++k) n += ((k * NW + wave) * 64 < NP) ? 1 : 0;
  return __builtin_amdgcn_readfirstlane(n);   // uniform: the waits below branch on it
}

// Wait until at most n of this wavefront's vector memory operations are
// outstanding. Loads return in issue order, so this completes every load
// issued before the n most recent ones.
__device__ __forceinline__ void wait_vm(int n) {
  switch (n) {
#define SAND_WAIT_VM(N) \
  case N: asm volatile("s_waitcnt vmcnt(" #N ")" ::: "memory"); break;
    SAND_WAIT_VM(1) SAND_WAIT_VM(2) SAND_WAIT_VM(3) SAND_WAIT_VM(4) SAND_WAIT_VM(5)
    SAND_WAIT_VM(6) SAND_WAIT_VM(7) SAND_WAIT_VM(8) SAND_WAIT_VM(9) SAND_WAIT_VM(10)
    SAND_WAIT_VM(11) SAND_WAIT_VM(12)
#undef SAND_WAIT_VM
    default: asm volatile("s_waitcnt vmcnt(0)" ::: "memory"); break;
  }
}

}  // namespace mfma
}  // namespace sand
