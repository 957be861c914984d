// Fused T-MLP evaluation on the matrix cores (gfx950): kernel templates,
// instantiated once per activation (tmlp_sine.hip, tmlp_finer.hip).
//
// One workgroup evaluates a tile of points that share an exit depth d
// (Sec. 3.4): hidden layers 1..d, each layer's tail, and the accumulated
// output y_d = t_1 + ... + t_d (Eq. 2), with tails of the product form of
// Eq. 3 where the model has them. Each result goes straight to its point's
// slot in the output.
//
// Data flow of one wavefront (one block of NQ points):
//  * Points are the N dimension of every product: Z_j = W_j H_{j-1}, with
//    W_j the A operand (from LDS) and H_{j-1} the B operand (registers).
//    BF16/FP16 use 32x32x16 MFMAs (32 points per wavefront, output blocks
//    of 32 units); FP32 uses 16x16x4 MFMAs (16 points, blocks of 16 units).
//    The packed weights' K order is permuted so that a layer's FP32
//    accumulators, after sine and conversion, are the next layer's B
//    operand as they stand: activations never leave registers.
//  * Layer 1 (K = 3 plus bias) keeps an FP32-accurate omega-scaled
//    argument in every precision: an FP32 MFMA with B = (x, y, z, 1) on the
//    FP32 path; on the BF16/FP16 paths BF16 MFMAs over three-way BF16
//    splits of weights and coordinates (six partial products, exact in
//    FP32). A linear first tail skips its zero second factor.
//  * Hidden-layer bias: one extra K step against a constant B = 1 (two
//    16-bit columns, high and low part, for BF16/FP16).
//  * Epilogue per element: hardware sine in revolutions (weights carry
//    omega/(2 pi)) of the activation's argument (SIREN: the accumulator
//    itself; FINER: scaled by 1 + |z|, two more vector instructions), two
//    FP32 FMAs for the two tail factors, pack. The lanes
//    holding disjoint units of one point are summed by cross-lane exchange.
//  * Weights stream through an LDS ring of PD + 2 slots, one output block
//    ("chunk") at a time: direct global-to-LDS loads of the next PD chunks
//    are in flight while chunk c feeds the MFMAs (PD = 1 by default).
//  * Software pipelining: each wavefront issues the MFMAs of block rb
//    together with the sine/tail epilogue of block rb-1; for BF16/FP16 the
//    block step is scheduled by hand, each MFMA carrying a share of that
//    epilogue and the A operands arriving in batches one batch ahead.
//  * Two wavefronts per SIMD: while one wavefront runs its sine/tail
//    epilogue on the vector ALU the other keeps the matrix core busy. By
//    default one workgroup of eight wavefronts per CU shares each weight
//    chunk among 256 points; SAND_FWD_WAVES=4 builds two independent
//    workgroups of four per CU instead (each with its own ring), which
//    measured slower on the 8x256 model (twice the weight traffic).
// The grid is persistent and strides over tiles, which the plan orders
// deepest bucket first; each tile's points and the first hidden chunk are
// fetched while the previous tile runs. Map-free dynamic exit runs in the
// same kernel (per-layer exit test, optional compaction of the points still
// running after a checkpoint layer into full tiles of a second launch).

#pragma once

#include "mfma_common.h"

#ifndef SAND_APF
#define SAND_APF 4
#endif

namespace sand {

namespace {

using namespace mfma;

// Tail partial sums of one 32-unit block for BF16/FP16: s0 += a0[unit(e)]
// h_e and s1 += a1[unit(e)] h_e over the lane's 16 registers, with each
// weight taken by a DPP row broadcast (row_newbcast:e) of the lane-indexed
// weights w0, w1, so the whole block reads 512 bytes of tail weights from
// LDS instead of 128 bytes per lane. The leading s_nop covers the wait
// states a DPP read needs after a VALU (or sine) write of its inputs, the
// trailing one those of whatever reads s0, s1 next.
__device__ __forceinline__ void tail_fma16(float& s0, float& s1, float w0, float w1,
                                           const float (&h)[16]) {
#define SAND_TAIL_E(E, R)                                                                   \
  "v_fmac_f32_dpp %0, %2, %" #R " row_newbcast:" #E " row_mask:0xf bank_mask:0xf\n\t"  \
  "v_fmac_f32_dpp %1, %3, %" #R " row_newbcast:" #E " row_mask:0xf bank_mask:0xf\n\t"
  asm("s_nop 1\n\t"
      SAND_TAIL_E(0, 4) SAND_TAIL_E(1, 5) SAND_TAIL_E(2, 6) SAND_TAIL_E(3, 7)
      SAND_TAIL_E(4, 8) SAND_TAIL_E(5, 9) SAND_TAIL_E(6, 10) SAND_TAIL_E(7, 11)
      SAND_TAIL_E(8, 12) SAND_TAIL_E(9, 13) SAND_TAIL_E(10, 14) SAND_TAIL_E(11, 15)
      SAND_TAIL_E(12, 16) SAND_TAIL_E(13, 17) SAND_TAIL_E(14, 18) SAND_TAIL_E(15, 19)
      "s_nop 1"
      : "+v"(s0), "+v"(s1)
      : "v"(w0), "v"(w1), "v"(h[0]), "v"(h[1]), "v"(h[2]), "v"(h[3]), "v"(h[4]), "v"(h[5]),
        "v"(h[6]), "v"(h[7]), "v"(h[8]), "v"(h[9]), "v"(h[10]), "v"(h[11]), "v"(h[12]),
        "v"(h[13]), "v"(h[14]), "v"(h[15]));
#undef SAND_TAIL_E
}

// One register's share of the BF16/FP16 tail sums: s0 += a0[unit(E)] h and
// s1 += a1[unit(E)] h, the weights broadcast from lane E of each 16-lane row
// (as in tail_fma16). The s_nop covers the wait states a DPP read of w0, w1
// needs after a VALU write of them.
template <int E>
__device__ __forceinline__ void tail_pair(float& s0, float& s1, float w0, float w1, float h);
#define SAND_TAIL_PAIR(E)                                                                       \
  template <>                                                                                   \
  __device__ __forceinline__ void tail_pair<E>(float& s0, float& s1, float w0, float w1,        \
                                               float h) {                                       \
    asm("s_nop 1\n\t"                                                                           \
        "v_fmac_f32_dpp %0, %2, %4 row_newbcast:" #E " row_mask:0xf bank_mask:0xf\n\t"           \
        "v_fmac_f32_dpp %1, %3, %4 row_newbcast:" #E " row_mask:0xf bank_mask:0xf"               \
        : "+v"(s0), "+v"(s1)                                                                    \
        : "v"(w0), "v"(w1), "v"(h));                                                            \
  }
SAND_TAIL_PAIR(0) SAND_TAIL_PAIR(1) SAND_TAIL_PAIR(2) SAND_TAIL_PAIR(3)
SAND_TAIL_PAIR(4) SAND_TAIL_PAIR(5) SAND_TAIL_PAIR(6) SAND_TAIL_PAIR(7)
SAND_TAIL_PAIR(8) SAND_TAIL_PAIR(9) SAND_TAIL_PAIR(10) SAND_TAIL_PAIR(11)
SAND_TAIL_PAIR(12) SAND_TAIL_PAIR(13) SAND_TAIL_PAIR(14) SAND_TAIL_PAIR(15)
#undef SAND_TAIL_PAIR

__device__ __forceinline__ void tail_pair_at(int e, float& s0, float& s1, float w0, float w1,
                                             float h) {
  switch (e) {   // e is a constant once the caller's loops are unrolled
    case 0: tail_pair<0>(s0, s1, w0, w1, h); break;
    case 1: tail_pair<1>(s0, s1, w0, w1, h); break;
    case 2: tail_pair<2>(s0, s1, w0, w1, h); break;
    case 3: tail_pair<3>(s0, s1, w0, w1, h); break;
    case 4: tail_pair<4>(s0, s1, w0, w1, h); break;
    case 5: tail_pair<5>(s0, s1, w0, w1, h); break;
    case 6: tail_pair<6>(s0, s1, w0, w1, h); break;
    case 7: tail_pair<7>(s0, s1, w0, w1, h); break;
    case 8: tail_pair<8>(s0, s1, w0, w1, h); break;
    case 9: tail_pair<9>(s0, s1, w0, w1, h); break;
    case 10: tail_pair<10>(s0, s1, w0, w1, h); break;
    case 11: tail_pair<11>(s0, s1, w0, w1, h); break;
    case 12: tail_pair<12>(s0, s1, w0, w1, h); break;
    case 13: tail_pair<13>(s0, s1, w0, w1, h); break;
    case 14: tail_pair<14>(s0, s1, w0, w1, h); break;
    default: tail_pair<15>(s0, s1, w0, w1, h); break;
  }
}

// tail_fma16 for a linear tail: the second factor (a1 = 0) is skipped.
__device__ __forceinline__ void tail_fma16_lin(float& s0, float w0, const float (&h)[16]) {
#define SAND_TAIL_L(E, R) \
  "v_fmac_f32_dpp %0, %1, %" #R " row_newbcast:" #E " row_mask:0xf bank_mask:0xf\n\t"
  asm("s_nop 1\n\t"
      SAND_TAIL_L(0, 2) SAND_TAIL_L(1, 3) SAND_TAIL_L(2, 4) SAND_TAIL_L(3, 5)
      SAND_TAIL_L(4, 6) SAND_TAIL_L(5, 7) SAND_TAIL_L(6, 8) SAND_TAIL_L(7, 9)
      SAND_TAIL_L(8, 10) SAND_TAIL_L(9, 11) SAND_TAIL_L(10, 12) SAND_TAIL_L(11, 13)
      SAND_TAIL_L(12, 14) SAND_TAIL_L(13, 15) SAND_TAIL_L(14, 16) SAND_TAIL_L(15, 17)
      "s_nop 1"
      : "+v"(s0)
      : "v"(w0), "v"(h[0]), "v"(h[1]), "v"(h[2]), "v"(h[3]), "v"(h[4]), "v"(h[5]), "v"(h[6]),
        "v"(h[7]), "v"(h[8]), "v"(h[9]), "v"(h[10]), "v"(h[11]), "v"(h[12]), "v"(h[13]),
        "v"(h[14]), "v"(h[15]));
#undef SAND_TAIL_L
}

// Epilogue of one output block: sine, tail partial sums, pack for the next layer.
// PACK = false: the layer is the tile's last, so its activations are not
// converted for a next layer. LIN: the tail is linear (s1 stays 0).
// BF16/FP16 form with the block's lane-indexed tail weights w0, w1 already
// in registers.
template <int PREC, int KS, bool PACK, bool LIN, int ACT>
__device__ __forceinline__ void epilogue16(float kf, float w0, float w1, int rb,
                                           const typename Tr<PREC>::Acc& acc,
                                           typename Tr<PREC>::V (&out)[KS], float& s0,
                                           float& s1) {
  using T = Tr<PREC>;
  float h[16];
#pragma unroll
  for (int e = 0; e < 16; ++e) h[e] = sin_rev(act_arg<ACT>(acc[e], kf));
  if constexpr (LIN)
    tail_fma16_lin(s0, w0, h);
  else
    tail_fma16(s0, s1, w0, w1, h);
  if constexpr (PACK) {
#pragma unroll
    for (int e = 0; e < 16; ++e) T::template put<KS>(out, rb, e, h[e]);
  }
}

template <int PREC, int KS, bool PACK, bool LIN, int ACT>
__device__ __forceinline__ void epilogue(float kf, const char* tails, int lane, int g, int rb,
                                         const typename Tr<PREC>::Acc& acc,
                                         typename Tr<PREC>::V (&out)[KS], float& s0, float& s1) {
  using T = Tr<PREC>;
  if constexpr (T::VB == 16) {
    const float w0 = ((const float*)tails)[lane];
    const float w1 = LIN ? 0.0f : ((const float*)tails)[64 + lane];
    epilogue16<PREC, KS, PACK, LIN, ACT>(kf, w0, w1, rb, acc, out, s0, s1);
  } else {
#pragma unroll
    for (int i = 0; i < T::NR / 4; ++i) {
      const f32x4 ta = T::tail_vec(tails, 0, i, g);
      const f32x4 tb = T::tail_vec(tails, 1, i, g);
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const int e = 4 * i + k;
        const float v = sin_rev(act_arg<ACT>(acc[e], kf));
        s0 = fmaf(ta[k], v, s0);
        if constexpr (!LIN) s1 = fmaf(tb[k], v, s1);
        if constexpr (PACK) T::template put<KS>(out, rb, e, v);
      }
    }
  }
}

// An output block's epilogue is pure register arithmetic, so the compiler
// may sink it past the following barriers and keep every block's
// accumulators and tail weights live at once (spilling to scratch). An
// empty asm that reads the block's results pins the epilogue in place.
template <int PREC, int KS, bool PACK = true>
__device__ __forceinline__ void pin_block(const typename Tr<PREC>::V (&out)[KS], int rb, float s0,
                                          float s1) {
  using T = Tr<PREC>;
  asm volatile("" ::"v"(s0), "v"(s1));
  if constexpr (!PACK) {
    return;
  } else if constexpr (T::VB == 16) {
    asm volatile("" ::"v"(out[2 * rb]), "v"(out[2 * rb + 1]));
  } else {
#pragma unroll
    for (int e = 0; e < T::NR; ++e) asm volatile("" ::"v"(out[4 * rb + e]));
  }
}

// Add tail t_j = u0 * u1 to the running output (u0, u1 its two factors,
// summed over the lanes that hold the point's units).
template <int PREC>
__device__ __forceinline__ float add_tail(float y, float s0, float s1, float c0, float c1,
                                          float* t = nullptr) {
  using T = Tr<PREC>;
  const float u0 = T::lane_sum(s0) + c0, u1 = T::lane_sum(s1) + c1;
  if (t) *t = u0 * u1;
  return fmaf(u0, u1, y);
}

// MFMA chain of one output block: bias + W_j h over all K steps, A operands
// from the LDS slot holding the block's chunk. The A operands are read PF
// steps ahead of their MFMA; the scheduling groups keep the compiler from
// sinking each read to its use, which would make every MFMA of the chain
// wait for a full LDS round trip.
template <int PREC, int WP>
__device__ __forceinline__ typename Tr<PREC>::Acc block_mma(
    const char* slot, int lane, const typename Tr<PREC>::V (&in)[Cfg<PREC, WP>::KS],
    const typename Tr<PREC>::V& bb) {
  using C = Cfg<PREC, WP>;
  using T = Tr<PREC>;
  using V = typename T::V;
  constexpr int NS = C::KS + 1;          // the bias step, then the KS weight steps
  constexpr int PF_WANT = WP > 256 ? 1 : SAND_APF;   // wider layers have no registers to spare
  constexpr int PF = NS < PF_WANT ? NS : PF_WANT;
  // the bias tile sits after the KS weight tiles in the chunk
  auto a_of = [&](int s) -> V {
    return *(const V*)(slot + ((s == 0 ? C::KS : s - 1) * 64 + lane) * T::VB);
  };
  V a[PF];
#pragma unroll
  for (int s = 0; s < PF; ++s) a[s] = a_of(s);
  typename T::Acc acc = {};
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const V cur = a[s % PF];
    if (s + PF < NS) a[s % PF] = a_of(s + PF);
    acc = T::mma(cur, s == 0 ? bb : in[s - 1], acc);
  }
  __builtin_amdgcn_sched_group_barrier(0x100, PF, 0);
#pragma unroll
  for (int s = 0; s < NS - PF; ++s) {
    __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
  }
  __builtin_amdgcn_sched_group_barrier(0x008, PF, 0);
  return acc;
}

// One block step of a BF16/FP16 hidden layer, scheduled by hand: the 17
// MFMAs of block rb (bias step first) each carry a share of block rb-1's
// epilogue (one sine, one tail pair, every other step one pack), so that a
// wavefront keeps the matrix core and the vector ALU busy together instead
// of alternating between an MFMA phase and a vector phase in step with the
// other wavefront of its SIMD. A operands arrive in batches of four, one
// batch ahead; each batch is awaited before the next is requested, so no
// wait covers a read issued just before it.
template <int PREC, int WP, bool EPI, int ACT>
__device__ __forceinline__ typename Tr<PREC>::Acc block_step16(
    float kf, const char* slot, const char* ptails, int lane, int rbp,
    const typename Tr<PREC>::V (&in)[Cfg<PREC, WP>::KS], const typename Tr<PREC>::V& bb,
    const typename Tr<PREC>::Acc& prev, typename Tr<PREC>::V (&out)[Cfg<PREC, WP>::KS],
    float& s0, float& s1) {
  using C = Cfg<PREC, WP>;
  using T = Tr<PREC>;
  using V = typename T::V;
  constexpr int NS = C::KS + 1;
  constexpr int NB = (NS + 3) / 4;
  auto a_of = [&](int s) -> V {
    return *(const V*)(slot + ((s == 0 ? C::KS : s - 1) * 64 + lane) * T::VB);
  };
  float w0 = 0.0f, w1 = 0.0f;
  if constexpr (EPI) {
    w0 = ((const float*)ptails)[lane];
    w1 = ((const float*)ptails)[64 + lane];
  }
  V a[2][4];
#pragma unroll
  for (int k = 0; k < 4; ++k)
    if (k < NS) a[0][k] = a_of(k);
  float h[16];
  typename T::Acc acc = {};
#pragma unroll
  for (int b = 0; b < NB; ++b) {
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (4 * b + k < NS) asm volatile("" ::"v"(a[b & 1][k]));
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (4 * (b + 1) + k < NS) a[(b + 1) & 1][k] = a_of(4 * (b + 1) + k);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int s = 4 * b + k;
      if (s < NS) {
        acc = T::mma(a[b & 1][k], s == 0 ? bb : in[s - 1], acc);
        if constexpr (EPI) {
          if (s < 16) h[s] = sin_rev(act_arg<ACT>(prev[s], kf));
          if (s >= 2 && s - 2 < 16) tail_pair_at(s - 2, s0, s1, w0, w1, h[s - 2]);
          if (s >= 2 && (s & 1) == 0 && s - 1 < 16) {
            T::template put<C::KS>(out, rbp, s - 2, h[s - 2]);
            T::template put<C::KS>(out, rbp, s - 1, h[s - 1]);
          }
        }
        __builtin_amdgcn_sched_barrier(0);
      }
    }
  }
  if constexpr (EPI) {
    // blocks with fewer than 16 MFMA steps finish their epilogue here
#pragma unroll
    for (int e = NS; e < 16; ++e) h[e] = sin_rev(act_arg<ACT>(prev[e], kf));
#pragma unroll
    for (int e = NS - 2; e < 16; ++e) tail_pair_at(e, s0, s1, w0, w1, h[e]);
#pragma unroll
    for (int e = (NS & ~1); e < 16; e += 2) {
      T::template put<C::KS>(out, rbp, e, h[e]);
      T::template put<C::KS>(out, rbp, e + 1, h[e + 1]);
    }
  }
  return acc;
}

#ifndef SAND_INTERLEAVE
#define SAND_INTERLEAVE 1
#endif

// One hidden layer: in -> out, streaming its RB chunks through an LDS ring of
// PD + 2 slots. Software-pipelined: the MFMAs of block rb are issued together
// with the (independent) sine/tail epilogue of block rb-1, so one
// wavefront keeps the matrix core and the vector ALU busy at once. Chunk c
// lives in slot c % (PD + 2); while block rb (chunk c) feeds the MFMAs and
// block rb-1's tail weights (chunk c-1) feed the epilogue, chunks c+1 .. c+PD
// stream into the other slots (PD chunks in flight hide the latency of the
// global-to-LDS copies). c is the tile's running chunk index, nc its chunk
// count.
template <int PREC, int WP, int ACT>
__device__ __forceinline__ float hidden_layer(float kf, float y, const char* __restrict__ hidden,
                                              char* ring,
                                              int wave, int lane, int g, int& c, int nc,
                                              const typename Tr<PREC>::V (&in)[Cfg<PREC, WP>::KS],
                                              typename Tr<PREC>::V (&out)[Cfg<PREC, WP>::KS],
                                              float c0, float c1, float& t) {
  using C = Cfg<PREC, WP>;
  using T = Tr<PREC>;
  using V = typename T::V;
  float s0 = 0.0f, s1 = 0.0f;
  const V bb = T::bias_b(g);
  const int lpc = chunk_loads<C::CH, C::NWF>(wave);
  typename T::Acc prev = {};
#pragma unroll
  for (int rb = 0; rb < C::RB; ++rb) {
    if (c + C::PD < nc)
      load_chunk<C::CH, C::NWF>(hidden + (size_t)(c + C::PD) * C::CH,
                               ring + ((c + C::PD) % C::NSLOT) * C::CH, wave, lane);
    typename T::Acc acc;
    if constexpr (T::VB == 16 && WP <= 256 && SAND_INTERLEAVE) {
      const char* ptails = ring + ((c + C::NSLOT - 1) % C::NSLOT) * C::CH + C::TAIL_OFF;
      if (rb > 0) {
        acc = block_step16<PREC, WP, true, ACT>(kf, ring + (c % C::NSLOT) * C::CH, ptails, lane,
                                                rb - 1, in, bb, prev, out, s0, s1);
        pin_block<PREC, C::KS>(out, rb - 1, s0, s1);
      } else {
        acc = block_step16<PREC, WP, false, ACT>(kf, ring + (c % C::NSLOT) * C::CH, ptails, lane, 0,
                                                 in, bb, prev, out, s0, s1);
      }
    } else {
      acc = block_mma<PREC, WP>(ring + (c % C::NSLOT) * C::CH, lane, in, bb);
      if (rb > 0) {
        epilogue<PREC, C::KS, true, false, ACT>(
            kf, ring + ((c + C::NSLOT - 1) % C::NSLOT) * C::CH + C::TAIL_OFF, lane, g, rb - 1, prev,
            out, s0, s1);
        pin_block<PREC, C::KS>(out, rb - 1, s0, s1);
      }
    }
    if (c + 1 < nc) {
      // chunk c+1 has landed once only the loads of chunks c+2 .. c+PD remain
      int later = 0;
#pragma unroll
      for (int k = 2; k <= C::PD; ++k) later += (c + k < nc) ? lpc : 0;
      wait_vm(later);
    }
    __syncthreads();
    prev = acc;
    ++c;
  }
  epilogue<PREC, C::KS, true, false, ACT>(
      kf, ring + ((c + C::NSLOT - 1) % C::NSLOT) * C::CH + C::TAIL_OFF, lane, g, C::RB - 1, prev,
      out, s0, s1);
  pin_block<PREC, C::KS>(out, C::RB - 1, s0, s1);
  return add_tail<PREC>(y, s0, s1, c0, c1, &t);
}

// Layer 1 and the partial sums of its tail, pipelined like the hidden
// layers: the MFMAs of block rb go with the epilogue of block rb-1. LIN: tail
// 1 is linear.
template <int PREC, int WP, bool PACK, bool LIN, int ACT>
__device__ __forceinline__ void layer1(float kf, const char* l1, int lane, int g, float px, float py,
                                       float pz, typename Tr<PREC>::V (&act)[Cfg<PREC, WP>::KS],
                                       float& s0, float& s1) {
  using C = Cfg<PREC, WP>;
  using T = Tr<PREC>;
  // The lane-indexed tail weights (BF16/FP16) are read up front and the A
  // operands one block ahead, so no LDS read is awaited right after its
  // issue.
  using L1V = typename T::L1V;
  float w0[C::RB], w1[C::RB];
  if constexpr (T::VB == 16) {
#pragma unroll
    for (int rb = 0; rb < C::RB; ++rb) {
      const float* tails = (const float*)(l1 + rb * C::L1C + T::L1S * T::L1AB);
      w0[rb] = tails[lane];
      w1[rb] = LIN ? 0.0f : tails[64 + lane];
    }
  }
  L1V a[2][T::L1S], b[T::L1S];
#pragma unroll
  for (int st = 0; st < T::L1S; ++st) {
    a[0][st] = T::l1_a(l1, st, lane);
    b[st] = T::l1_b(st, g, px, py, pz);
  }
  typename T::Acc prev = {};
#pragma unroll
  for (int rb = 0; rb <= C::RB; ++rb) {
    typename T::Acc acc = {};
    if (rb < C::RB) {
      if (rb + 1 < C::RB) {
#pragma unroll
        for (int st = 0; st < T::L1S; ++st)
          a[(rb + 1) & 1][st] = T::l1_a(l1 + (rb + 1) * C::L1C, st, lane);
      }
#pragma unroll
      for (int st = 0; st < T::L1S; ++st) acc = T::mma1(a[rb & 1][st], b[st], acc);
    }
    // both MFMAs of block rb go out before block rb-1's epilogue reads its
    // own (older) results, so no read waits on an MFMA still in flight
    __builtin_amdgcn_sched_barrier(0);
    if (rb > 0) {
      if constexpr (T::VB == 16)
        epilogue16<PREC, C::KS, PACK, LIN, ACT>(kf, w0[rb - 1], w1[rb - 1], rb - 1, prev, act, s0,
                                                s1);
      else
        epilogue<PREC, C::KS, PACK, LIN, ACT>(kf, l1 + (rb - 1) * C::L1C + T::L1S * T::L1AB, lane,
                                              g, rb - 1, prev, act, s0, s1);
      pin_block<PREC, C::KS, PACK>(act, rb - 1, s0, s1);
    }
    prev = acc;
  }
}

// Decode tile `tile` of a plan: exit depth, first permutation slot, count.
// tile_end[dd] falls as dd grows and is 0 beyond the deepest depth, so the
// depth is the number of dd >= 1 with tile < tile_end[dd]: independent
// reads, no dependent search.
template <int Q>
__device__ __forceinline__ void decode_tile(const Plan* plan, int L, int64_t tile, int& d,
                                            int64_t& start, int64_t& cnt) {
  d = 0;
#pragma unroll
  for (int dd = 1; dd < kBuckets; ++dd) d += (int)(tile < plan->tile_end[dd]);
  if (d < 1) d = 1;
  const int64_t local = tile - plan->tile_end[d + 1];
  start = plan->start[d] + local * Q;
  cnt = plan->count[d] - local * Q;
  if (cnt > Q) cnt = Q;
}

// Hidden layers j0..d of a tile. Layer j reads actA and writes actB when j
// is even, the reverse when it is odd (layer 1 writes actA). `after(j, y_j,
// t_j, out)` sees each layer's output (out: its packed activations) and
// returns false to stop the tile. ODD_START: j0 is odd (a resumed tile).
template <int PREC, int WP, int ACT, bool ODD_START, class After>
__device__ __forceinline__ void run_layers(const ModelArgs& M, int j0, int d, float y,
                                           const char* hidden, char* ring, int wave, int lane,
                                           int g, int& c, int nc,
                                           typename Tr<PREC>::V (&actA)[Cfg<PREC, WP>::KS],
                                           typename Tr<PREC>::V (&actB)[Cfg<PREC, WP>::KS],
                                           After after) {
  using V = typename Tr<PREC>::V;
  constexpr int KS = Cfg<PREC, WP>::KS;
  // layers j0, j0 + 2, ... read `p` and write `q`; the others the reverse
  V (&p)[KS] = ODD_START ? actB : actA;
  V (&q)[KS] = ODD_START ? actA : actB;
  float t;
  for (int j = j0; j <= d; j += 2) {
    y = hidden_layer<PREC, WP, ACT>(M.kf[1], y, hidden, ring, wave, lane, g, c, nc, p, q,
                                    M.c0[j - 1], M.c1[j - 1], t);
    if (!after(j, y, t, q) || j + 1 > d) break;
    y = hidden_layer<PREC, WP, ACT>(M.kf[1], y, hidden, ring, wave, lane, g, c, nc, q, p, M.c0[j],
                                    M.c1[j], t);
    if (!after(j + 1, y, t, p)) break;
  }
}

// Write the records of this wavefront's points that are still running after
// layer j (spill arena of compacted dynamic exit); `out` holds layer j's
// packed output. One atomic per wavefront reserves the records.
template <int PREC, int WP>
__device__ __forceinline__ void spill_points(const DynSpill& sp, bool running, int gi, float y,
                                             int lane, int g,
                                             const typename Tr<PREC>::V (&out)[Cfg<PREC, WP>::KS]) {
  using C = Cfg<PREC, WP>;
  using T = Tr<PREC>;
  using V = typename T::V;
  const int col = T::col(lane);
  const uint64_t m = __ballot(running && g == 0);   // group-0 lanes are columns 0..NQ-1
  int base = 0;
  if (lane == 0 && m != 0ull) base = atomicAdd(sp.count, __popcll(m));
  base = __shfl(base, 0);
  const int rank = __popcll(m & (col == 0 ? 0ull : (~0ull >> (64 - col))));
  const int64_t r = (int64_t)base + rank;
  if (!running || r >= sp.cap) return;
  char* rec = sp.arena + r * C::REC;
  if (g == 0) {
    ((int*)rec)[0] = gi;
    ((float*)rec)[1] = y;
  }
  V* dst = (V*)(rec + 16 + g * C::KS * T::VB);
#pragma unroll
  for (int s = 0; s < C::KS; ++s) dst[s] = out[s];
}

// Evaluate one tile of exit depth d. This lane's point is gi (< 0: none)
// at (px, py, pz); every lane of the same column holds the same point.
// Returns whether this lane writes the point's result, yout, to the output
// (left to the caller, which can first settle its own loads: a wait placed
// after a conditional store must assume the store is still outstanding).
template <int PREC, int WP, int ACT>
__device__ __forceinline__ bool run_tile(const ModelArgs& M, float& yout, int d,
                                         int gi, float px, float py, float pz, char* ring,
                                         const char* l1, int lane, int wave,
                                         float* __restrict__ y_all, float dyn_r,
                                         uint8_t* __restrict__ depth_out, const DynSpill& sp) {
  using C = Cfg<PREC, WP>;
  using T = Tr<PREC>;
  using V = typename T::V;
  const int g = T::grp(lane);
  const char* hidden = M.chunks + C::L1B;
  const bool ok = gi >= 0;

  // The first PD hidden chunks stream into the ring while layer 1 runs (layer
  // 1 reads only its own LDS region; every ring slot is free at a tile's
  // start).
  const int nc = (d - 1) * C::RB;
#pragma unroll
  for (int k = 0; k < C::PD; ++k)
    if (k < nc) load_chunk<C::CH, C::NWF>(hidden + (size_t)k * C::CH, ring + k * C::CH, wave, lane);

  V actA[C::KS], actB[C::KS];
  float s0 = 0.0f, s1 = 0.0f;
  const bool lin1 = (M.lin_mask & 1u) != 0;
  if (d > 1) {
    if (lin1)
      layer1<PREC, WP, true, true, ACT>(M.kf[0], l1, lane, g, px, py, pz, actA, s0, s1);
    else
      layer1<PREC, WP, true, false, ACT>(M.kf[0], l1, lane, g, px, py, pz, actA, s0, s1);
  } else {
    if (lin1)
      layer1<PREC, WP, false, true, ACT>(M.kf[0], l1, lane, g, px, py, pz, actA, s0, s1);
    else
      layer1<PREC, WP, false, false, ACT>(M.kf[0], l1, lane, g, px, py, pz, actA, s0, s1);
  }
  float y = add_tail<PREC>(0.0f, s0, s1, M.c0[0], M.c1[0]);
  // every accumulated output y_j, for building a depth map (Eq. 5)
  float* yrow = (y_all && g == 0 && ok) ? y_all + (int64_t)gi * M.L : nullptr;
  if (yrow) yrow[0] = y;

  int c = 0;
  if (nc > 0) {
    const int lpc = chunk_loads<C::CH, C::NWF>(wave);
    int later = 0;   // loads of chunks 1 .. PD-1
#pragma unroll
    for (int k = 1; k < C::PD; ++k) later += (k < nc) ? lpc : 0;
    wait_vm(later);
    __syncthreads();
  }
  // Map-free early exit (dyn_r > 0): a point's output is frozen after the
  // first layer j >= 2 whose tail t_j is below dyn_r in magnitude; the
  // workgroup stops once none of its points is still running. With
  // compaction (sp.layer), the points still running after layer sp.layer
  // leave as records and the tile stops.
  bool alive = ok, spilled = false;
  int dexit = d;
  auto after_layer = [&](int j, float yn, float t, const V (&out)[C::KS]) {
    if (dyn_r > 0.0f) {
      if (alive) {
        y = yn;
        if (fabsf(t) < dyn_r) {
          alive = false;
          dexit = j;
        }
      }
      if (j == sp.layer && j < d) {
        spill_points<PREC, WP>(sp, alive, gi, y, lane, g, out);
        spilled = alive;
        alive = false;
        return false;
      }
      return __syncthreads_or(alive ? 1 : 0) != 0;
    }
    y = yn;
    if (yrow) yrow[j - 1] = y;
    return true;
  };
  run_layers<PREC, WP, ACT, false>(M, 2, d, y, hidden, ring, wave, lane, g, c, nc, actA, actB,
                                   after_layer);
  const bool done = ok && !spilled;
  if (depth_out && g == 0 && done) depth_out[gi] = (uint8_t)(dyn_r > 0.0f ? dexit : d);
  // the last epilogue read a ring slot the next tile's first load may reuse,
  // and an early exit can leave chunk copies in flight
  if (nc > 0) {
    wait_chunk();
    __syncthreads();
  }
  yout = y;
  return g == 0 && done;
}

// A resumed tile of compacted dynamic exit: up to Q records, each run from
// layer j0 = spill layer + 1 to d with the exit test. This lane's record is
// ri (< 0: none). ODD: j0 is odd.
template <int PREC, int WP, int ACT, bool ODD>
__device__ __forceinline__ void resume_tile(const ModelArgs& M, float* __restrict__ sdf, int d,
                                            const DynSpill& sp, int ri, char* ring, int lane,
                                            int wave, float dyn_r,
                                            uint8_t* __restrict__ depth_out) {
  using C = Cfg<PREC, WP>;
  using T = Tr<PREC>;
  using V = typename T::V;
  const int g = T::grp(lane);
  const char* hidden = M.chunks + C::L1B;
  const int j0 = sp.layer + 1;
  V actA[C::KS], actB[C::KS];
  int gi = -1;
  float y = 0.0f;
  const char* rec = sp.arena + (int64_t)(ri < 0 ? 0 : ri) * C::REC;
  const V* src = (const V*)(rec + 16 + g * C::KS * T::VB);
  if (ri >= 0) {
    gi = ((const int*)rec)[0];
    y = ((const float*)rec)[1];
  }
  const bool ok = gi >= 0;
  // chunks of layers j0..d: absolute chunk indices c0 .. nc-1, chunk c in
  // ring slot c % NSLOT as in run_tile
  const int c0 = (j0 - 2) * C::RB, nc = (d - 1) * C::RB;
  int c = c0;
#pragma unroll
  for (int k = 0; k < C::PD; ++k)
    if (c0 + k < nc)
      load_chunk<C::CH, C::NWF>(hidden + (size_t)(c0 + k) * C::CH,
                                ring + ((c0 + k) % C::NSLOT) * C::CH, wave, lane);
  if (c0 < nc) {
    const int lpc = chunk_loads<C::CH, C::NWF>(wave);
    int later = 0;
#pragma unroll
    for (int k = 1; k < C::PD; ++k) later += (c0 + k < nc) ? lpc : 0;
    wait_vm(later);
    __syncthreads();
  }
  bool alive = ok;
  int dexit = d;
  auto after_layer = [&](int j, float yn, float t, const V (&)[C::KS]) {
    if (alive) {
      y = yn;
      if (fabsf(t) < dyn_r) {
        alive = false;
        dexit = j;
      }
    }
    return __syncthreads_or(alive ? 1 : 0) != 0;
  };
  // the record's activations are layer j0's input: actB when j0 is odd
  V (&in)[C::KS] = ODD ? actB : actA;
#pragma unroll
  for (int s = 0; s < C::KS; ++s) in[s] = ri >= 0 ? src[s] : V{};
  run_layers<PREC, WP, ACT, ODD>(M, j0, d, y, hidden, ring, wave, lane, g, c, nc, actA, actB,
                                 after_layer);
  if (depth_out && g == 0 && ok) depth_out[gi] = (uint8_t)dexit;
  if (c0 < nc) {
    wait_chunk();
    __syncthreads();
  }
  if (g == 0 && ok) sdf[gi] = y;
}

template <int PREC, int WP>
__device__ __forceinline__ void load_layer1(const ModelArgs& M, char* l1, int tid) {
  using C = Cfg<PREC, WP>;
  for (int i = tid; i < C::L1B / 16; i += C::NTF) ((uint4*)l1)[i] = ((const uint4*)M.chunks)[i];
}

// A workgroup's walk over its tiles, in increasing order. The plan puts
// deeper buckets first, so along the walk the exit depth only falls and a
// bucket's bounds are read (from the workgroup's LDS copy of the plan) only
// when the walk enters it. Bucket d holds tiles [lo, hi).
struct TileWalk {
  int d;
  int64_t lo, hi, start, count;
};

// Exit depth of tile `tile` and this lane's point in it (-1: none; qi is
// the lane's slot in the tile). Successive calls ask for increasing tiles.
template <int Q>
__device__ __forceinline__ int tile_point(const QueryArgs& a, const Plan& plan, TileWalk& w,
                                          int64_t total, int64_t tile, int qi, int& d) {
  int64_t start, cnt;
  if (tile >= total) {
    d = 1;
    return -1;
  }
  if (a.plan) {
    // ends by bucket 1 at the latest: tile < total = tile_end[1]
    while (tile >= w.hi && w.d > 1) {
      --w.d;
      w.lo = w.hi;
      w.hi = plan.tile_end[w.d];
      w.start = plan.start[w.d];
      w.count = plan.count[w.d];
    }
    d = w.d;
    const int64_t local = tile - w.lo;
    start = w.start + local * Q;
    cnt = w.count - local * Q;
    if (cnt > Q) cnt = Q;
  } else {
    d = a.full_depth;
    start = tile * Q;
    cnt = a.n - start < Q ? a.n - start : Q;
  }
  if (qi >= cnt) return -1;
  return a.perm ? a.perm[start + qi] : (int)(start + qi);
}

__device__ __forceinline__ void point_coords(const float* __restrict__ xyz, int gi, float& x,
                                             float& y, float& z) {
  x = y = z = 0.0f;
  if (gi >= 0) {
    const float* p = xyz + 3 * (int64_t)gi;
    x = p[0];
    y = p[1];
    z = p[2];
  }
}

// Persistent: workgroup b runs tiles b, b + G, b + 2G, ... (G = grid size).
// Point fetches are pipelined across tiles: while tile t runs, the
// coordinates of tile t + G and the permutation entries of tile t + 2G are
// in flight, so no tile starts on a dependent chain of global loads.
template <int PREC, int WP, int ACT>
__global__ __launch_bounds__((Cfg<PREC, WP>::NTF)) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_tmlp(QueryArgs a) {
  using C = Cfg<PREC, WP>;
  using T = Tr<PREC>;
  constexpr int Q = C::QF;
  __shared__ __attribute__((aligned(16))) char lds[C::LDS];
  __shared__ Plan splan;
  char* ring = lds;
  char* l1 = lds + C::NSLOT * C::CH;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  load_layer1<PREC, WP>(a.m, l1, tid);
  if (a.plan)
    for (int i = tid; i < (int)(sizeof(Plan) / 8); i += C::NTF)
      ((int64_t*)&splan)[i] = ((const int64_t*)a.plan)[i];
  __syncthreads();
  const Plan& plan = splan;
  const int64_t total = a.plan ? plan.total_tiles : (a.n + Q - 1) / Q;
  const int64_t G = gridDim.x;
  const int qi = wave * T::NQ + T::col(lane);
  int64_t tile = blockIdx.x;
  // buckets above L are empty: the walk starts past the deepest one
  TileWalk walk{a.m.L + 1, 0, 0, 0, 0};
  int d, d_next;
  int gi = tile_point<Q>(a, plan, walk, total, tile, qi, d);
  int gi_next = tile_point<Q>(a, plan, walk, total, tile + G, qi, d_next);
  float px, py, pz;
  point_coords(a.xyz, gi, px, py, pz);
  // Consume the first loads here: otherwise the loop entry merges their
  // pending state with the loop's and the first tile's layer-1 operands wait
  // for every load issued in the loop body, prefetches included.
  asm volatile("" ::"v"(gi_next), "v"(px), "v"(py), "v"(pz));
  for (; tile < total; tile += G) {
    int d_after;
    const int gi_after = tile_point<Q>(a, plan, walk, total, tile + 2 * G, qi, d_after);
    float nx, ny, nz;
    point_coords(a.xyz, gi_next, nx, ny, nz);
    float y;
    const bool st = run_tile<PREC, WP, ACT>(a.m, y, d, gi, px, py, pz, ring, l1, lane, wave,
                                            a.y_all, a.dyn_r, a.depth_out, a.spill);
    // The next tiles' prefetched coordinates and permutation entries have
    // had a whole tile to land: take them before the store, so that moving
    // them into place at the loop's end needs no wait for the store.
    asm volatile("" ::"v"(gi_after), "v"(nx), "v"(ny), "v"(nz));
    if (st) a.sdf[gi] = y;
    d = d_next;
    gi = gi_next;
    px = nx;
    py = ny;
    pz = nz;
    d_next = d_after;
    gi_next = gi_after;
  }
}

// Several queries (possibly of different models of the same padded width)
// in one persistent launch: tile t belongs to the last query whose first
// tile is <= t. Layer-1 weights are reloaded into LDS when the model changes.
template <int PREC, int WP, int ACT>
__global__ __launch_bounds__((Cfg<PREC, WP>::NTF)) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_tmlp_batch(BatchArgs a) {
  using C = Cfg<PREC, WP>;
  constexpr int Q = C::QF;
  __shared__ __attribute__((aligned(16))) char ring[C::NSLOT * C::CH];
  __shared__ __attribute__((aligned(16))) char l1[C::L1B];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  uint64_t cur = 0;   // address of the model whose layer 1 is in LDS
  const int64_t total = *a.total_tiles;
  for (int64_t tile = blockIdx.x; tile < total; tile += gridDim.x) {
    int lo = 0, hi = a.nreq - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (a.reqs[mid].tile0 <= tile) lo = mid; else hi = mid - 1;
    }
    const BatchReq& q = a.reqs[lo];
    const ModelArgs& M = *q.model;
    const uint64_t key = (uint64_t)(uintptr_t)q.model;
    if (key != cur) {
      __syncthreads();   // every wavefront is done with the previous layer-1 copy
      load_layer1<PREC, WP>(M, l1, tid);
      __syncthreads();
      cur = key;
    }
    int d;
    int64_t start, cnt;
    decode_tile<Q>(&q.plan, q.L, tile - q.tile0, d, start, cnt);
    const int qi = wave * Tr<PREC>::NQ + Tr<PREC>::col(lane);
    const int gi = qi < cnt ? q.perm[start + qi] : -1;
    float px, py, pz;
    point_coords(q.xyz, gi, px, py, pz);
    float y;
    if (run_tile<PREC, WP, ACT>(M, y, d, gi, px, py, pz, ring, l1, lane, wave, nullptr, 0.0f,
                                nullptr, DynSpill{}))
      q.sdf[gi] = y;
  }
}

// Second launch of compacted dynamic exit: persistent over the tiles of the
// records the spilling launch wrote (their count is read on the device).
template <int PREC, int WP, int ACT, bool ODD>
__global__ __launch_bounds__((Cfg<PREC, WP>::NTF)) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_tmlp_resume(QueryArgs a) {
  using C = Cfg<PREC, WP>;
  using T = Tr<PREC>;
  constexpr int Q = C::QF;
  __shared__ __attribute__((aligned(16))) char ring[C::NSLOT * C::CH];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  int64_t count = *a.spill.count;
  if (count > a.spill.cap) count = a.spill.cap;
  const int64_t total = (count + Q - 1) / Q;
  const int qi = wave * T::NQ + T::col(lane);
  for (int64_t tile = blockIdx.x; tile < total; tile += gridDim.x) {
    const int64_t ri = tile * Q + qi;
    resume_tile<PREC, WP, ACT, ODD>(a.m, a.sdf, a.full_depth, a.spill, ri < count ? (int)ri : -1,
                                    ring, lane, wave, a.dyn_r, a.depth_out);
  }
}

template <int PREC, int WP, int ACT>
hipError_t launch_one(const QueryArgs& a, int num_cu, hipStream_t s) {
  using C = Cfg<PREC, WP>;
  int64_t grid = (int64_t)num_cu * C::WGF;
  if (!a.plan) {
    const int64_t tiles = (a.n + C::QF - 1) / C::QF;
    if (tiles < grid) grid = tiles;
  }
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL((k_tmlp<PREC, WP, ACT>), dim3((unsigned)grid), dim3(C::NTF), 0, s, a);
  return hipGetLastError();
}

template <int PREC, int WP, int ACT>
hipError_t launch_resume_one(const QueryArgs& a, int num_cu, hipStream_t s) {
  using C = Cfg<PREC, WP>;
  if ((a.spill.layer + 1) & 1)
    hipLaunchKernelGGL((k_tmlp_resume<PREC, WP, ACT, true>), dim3((unsigned)(num_cu * C::WGF)),
                       dim3(C::NTF), 0, s, a);
  else
    hipLaunchKernelGGL((k_tmlp_resume<PREC, WP, ACT, false>), dim3((unsigned)(num_cu * C::WGF)),
                       dim3(C::NTF), 0, s, a);
  return hipGetLastError();
}

template <int PREC, int WP, int ACT>
hipError_t launch_batch_one(const BatchArgs& a, int num_cu, hipStream_t s) {
  hipLaunchKernelGGL((k_tmlp_batch<PREC, WP, ACT>),
                     dim3((unsigned)(num_cu * Cfg<PREC, WP>::WGF)), dim3(Cfg<PREC, WP>::NTF), 0,
                     s, a);
  return hipGetLastError();
}

// What: 0 a query, 1 a resumed launch of compacted dynamic exit, 2 a batch.
template <int PREC, int ACT>
hipError_t launch_width(int what, int WP, const QueryArgs* q, const BatchArgs* b, int num_cu,
                        hipStream_t s) {
#define SAND_WIDTH(W)                                                   \
  case W:                                                               \
    return what == 0   ? launch_one<PREC, W, ACT>(*q, num_cu, s)        \
           : what == 1 ? launch_resume_one<PREC, W, ACT>(*q, num_cu, s) \
                       : launch_batch_one<PREC, W, ACT>(*b, num_cu, s);
  switch (WP) {
    SAND_WIDTH(64) SAND_WIDTH(128) SAND_WIDTH(256) SAND_WIDTH(352)
    default: return hipErrorInvalidValue;
  }
#undef SAND_WIDTH
}

}  // namespace

template <int ACT>
hipError_t launch_tmlp_act(int what, int prec, int WP, const QueryArgs* q, const BatchArgs* b,
                           int num_cu, hipStream_t s) {
  if (prec == PREC_FP32) return launch_width<PREC_FP32, ACT>(what, WP, q, b, num_cu, s);
  if (prec == PREC_BF16) return launch_width<PREC_BF16, ACT>(what, WP, q, b, num_cu, s);
  return launch_width<PREC_FP16, ACT>(what, WP, q, b, num_cu, s);
}

}  // namespace sand
