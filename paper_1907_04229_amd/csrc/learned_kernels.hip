// Device kernels of the learned second stage (included once by cptr.hip).
//
// A message-passing network on the 7-point cell graph stands in for the ILU(0)
// second stage (it is not in the paper).  Hidden width 64, 3 layers:
//   r = D^{-1} b1, s_k = RMS over cells of r_k (per unknown), u_k = r_k / s_k
//   h0 = W_in u
//   e_{i,d} = S^{-1} D_i^{-1} A_{i,nbr(i,d)} S, S = diag(s) (scaled unknowns)
//   g_{i,d} = W_e e_{i,d};  m_i = sum_d g_{i,d} * h_{nbr(i,d)}
//   a_i = W_s h_i + W_m m_i + b;  h_i <- h_i + relu(a_i)
//   z2_k = s_k (u_k + (W_out h3)_k)
// The dense products (edge gating, W_s h, W_m m and the weight gradients,
// which reduce over cells) run on v_mfma_f32_16x16x16_bf16 with FP32
// accumulation: one wavefront per tile of 16 cells.  Activations are kept in
// FP32 in memory and rounded to BF16 only as MFMA operands.
//
// MFMA 16x16x16 operand layout (lane l = 0..63, q = 0..3):
//   A (16 x 16):  lane holds A[l % 16][4 (l / 16) + q]
//   B (16 x 16):  lane holds B[4 (l / 16) + q][l % 16]
//   D (16 x 16):  lane holds D[4 (l / 16) + q][l % 16]   (q = register)
#pragma once

#include <type_traits>

namespace cptr {

constexpr int kHid = 64;   // hidden width
constexpr int kDir = 6;    // neighbours on the 7-point stencil
constexpr int kEdge = 16;  // edge features padded to the MFMA depth (nv^2 <= 16)

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short f2bf(float f) {  // round to nearest even (v_cvt_pk_bf16_f32)
  return __builtin_bit_cast(short, (__bf16)f);
}

__device__ __forceinline__ f32x4 mfma16(bf16x4 a, bf16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// 16x16x32 BF16 MFMA (gfx950): A 16 x 32, lane holds A[l % 16][8 (l / 16) + j];
// B 32 x 16, lane holds B[8 (l / 16) + j][l % 16]; D as for 16x16x16.
typedef short bf16x8 __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
__device__ __forceinline__ f32x4 mfma32(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a), __builtin_bit_cast(bf16x8_t, b),
                                                 c, 0, 0, 0);
}
__device__ __forceinline__ bf16x8 cat8(bf16x4 x, bf16x4 y) {
  return __builtin_shufflevector(x, y, 0, 1, 2, 3, 4, 5, 6, 7);
}

__device__ __forceinline__ bf16x4 load_bf4(const short *p) {
  return *reinterpret_cast<const bf16x4 *>(p);
}

typedef __bf16 bf16x4_t __attribute__((ext_vector_type(4)));
__device__ __forceinline__ bf16x4 cvt4(float a, float b, float c, float d) {
  return __builtin_bit_cast(bf16x4, __builtin_convertvector((f32x4{a, b, c, d}), bf16x4_t));
}

// edge features in the scaled unknowns: e[r][c] * s_c / s_r for the four
// consecutive flattened entries k0..k0+3 (k = r NV + c; padding stays zero)
template <int NV>
__device__ __forceinline__ bf16x4 scale_edge4(bf16x4 e, int k0, const float *__restrict__ s) {
  bf16x4 o;
#pragma unroll
  for (int q = 0; q < 4; q++) {
    const int k = k0 + q;
    float v = __uint_as_float(uint32_t((unsigned short)e[q]) << 16);
    if (k < NV * NV) {
      const float sr = s[k / NV];
      v *= sr > 0.f ? s[k % NV] / sr : 0.f;
    } else {
      v = 0.f;
    }
    o[q] = f2bf(v);
  }
  return o;
}

template <int NV>
__device__ __forceinline__ float edge_factor(int k, const float *__restrict__ s) {
  if (k >= NV * NV) return 0.f;
  const float sr = s[k / NV];
  return sr > 0.f ? s[k % NV] / sr : 0.f;
}

// r = D^{-1} b1 (b1 of type BT), partial sums of r_k^2 per workgroup and unknown
template <int NV, typename BT>
__global__ void __launch_bounds__(kBlock) k_lrn_input(int n, const float *__restrict__ dinv,
                                                      const BT *__restrict__ b1,
                                                      float *__restrict__ r,
                                                      double *__restrict__ part) {
  __shared__ double sh[kBlock / 64][NV];
  const int i = blockIdx.x * kBlock + threadIdx.x;
  double acc[NV];
#pragma unroll
  for (int q = 0; q < NV; q++) acc[q] = 0.0;
  if (i < n) {
    float b[NV];
#pragma unroll
    for (int c = 0; c < NV; c++) b[c] = float(b1[(size_t)i * NV + c]);
#pragma unroll
    for (int q = 0; q < NV; q++) {
      float s = 0.f;
#pragma unroll
      for (int c = 0; c < NV; c++) s += dinv[((size_t)i * NV + q) * NV + c] * b[c];
      r[(size_t)i * NV + q] = s;
      acc[q] = double(s) * s;
    }
  }
#pragma unroll
  for (int q = 0; q < NV; q++) {
    const double v = wave_sum(acc[q]);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6][q] = v;
  }
  __syncthreads();
  if (threadIdx.x < NV) {
    double t = 0.0;
    for (int w = 0; w < kBlock / 64; w++) t += sh[w][threadIdx.x];
    part[(size_t)blockIdx.x * NV + threadIdx.x] = t;
  }
}

// s_k = sqrt(sum_k / n) from the partials (one workgroup per unknown, fixed order)
template <int NV>
__global__ void __launch_bounds__(kBlock) k_lrn_scale(const double *__restrict__ part, int nb,
                                                      double count, float *__restrict__ s_out) {
  __shared__ double sh[kBlock / 64];
  const int k = blockIdx.x;
  double acc = 0.0;
  for (int b = threadIdx.x; b < nb; b += kBlock) acc += part[(size_t)b * NV + k];
  acc = wave_sum(acc);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kBlock / 64; w++) t += sh[w];
    s_out[k] = float(sqrt(t / count));
  }
}

// Read-out of the last layer: z_k = r_k + s_k (W_out h3)_k, written as the
// FP64 vector `z2_out` when given, otherwise as z = z2 + x1 (the full
// two-stage result, x1 holding only the p and T components dp, dT) in the
// output type ZT through the apply slots.
template <typename ZT, typename XT>
struct LrnOut {
  const float *W_out;
  int ip, iT;
  const XT *dp, *dT;
  const ApplySlots *slots;
  double *z2_out;
};

// The output column of the slots, read once per workgroup (a store through
// slots->z in the tile loop would reload the pointer after every store)
template <bool LAST, typename ZT, typename XT>
__device__ __forceinline__ ZT *lrn_zout(const LrnOut<ZT, XT> &out) {
  return LAST && !out.z2_out && out.slots ? reinterpret_cast<ZT *>(as_global(out.slots)->z) : nullptr;
}

__device__ __forceinline__ f32x4 load_f4(const float *p) { return *reinterpret_cast<const f32x4 *>(p); }
__device__ __forceinline__ void store_f4(float *p, f32x4 v) { *reinterpret_cast<f32x4 *>(p) = v; }
__device__ __forceinline__ float bf2f(short b) { return __uint_as_float(uint32_t((unsigned short)b) << 16); }

// activations in memory: FP32, or BF16 (short) where only the forward pass needs them
__device__ __forceinline__ f32x4 load_h4(const float *p) { return load_f4(p); }
__device__ __forceinline__ f32x4 load_h4(const short *p) {
  const bf16x4 v = load_bf4(p);
  return f32x4{bf2f(v[0]), bf2f(v[1]), bf2f(v[2]), bf2f(v[3])};
}
__device__ __forceinline__ void store_h4(float *p, f32x4 v) { store_f4(p, v); }
__device__ __forceinline__ void store_h4(short *p, f32x4 v) {
  *reinterpret_cast<bf16x4 *>(p) = cvt4(v[0], v[1], v[2], v[3]);
}

// Channel map of the layer kernel: register slot t (0..3) of a lane in lane
// group lg holds the four consecutive hidden channels lch(t, lg) .. + 3.  With
// this order the slots 2 ks and 2 ks + 1 of a lane are exactly the eight
// consecutive channels 32 ks + 8 lg .. + 7 that a 16x16x32 B operand takes;
// activations stay in channel order in memory.
__device__ __forceinline__ int lch(int t, int lg) { return 32 * (t >> 1) + 8 * lg + 4 * (t & 1); }

// Offset of channel ch of a cell's activations.  FP32 activations (training)
// are rows of 64 channels; the BF16 activations of the forward pass are in
// tile order: for tile t = cell / 16, half ks = ch / 32 and lane group
// g = (ch % 32) / 8, the eight channels of the 16 cells are 16 x 8
// consecutive BF16, so a wave's load of one half is 1 KB contiguous (the
// arrays are padded to whole tiles).
__device__ __forceinline__ size_t h_off(const float *, int cell, int ch) {
  return (size_t)cell * kHid + ch;
}
// (32-bit offsets: 64 n < 2^32 for the grids this library takes; they keep
// the address arithmetic in single registers)
__device__ __forceinline__ uint32_t h_off(const short *, int cell, int ch) {
  return (uint32_t)(cell >> 4) * 1024u + (uint32_t)(ch >> 5) * 512u + (uint32_t)((ch >> 3) & 3) * 128u +
         (uint32_t)(cell & 15) * 8u + (uint32_t)(ch & 7);
}

// Neighbour activations as loaded (before conversion): BF16 or FP32 rows of
// the lane's 16 channels, or, for the first layer, the nv values of r from
// which h0 = W_in (r / s) is formed.
template <typename HT, int NV, bool FIRST>
struct RawAct;
template <int NV>
struct RawAct<short, NV, false> {
  struct type { bf16x4 v[4]; };
  static __device__ __forceinline__ type load(int cell, int lg, const short *h, const float *) {
    type o;
#pragma unroll
    for (int t = 0; t < 4; t++) o.v[t] = load_bf4(h + h_off(h, cell, lch(t, lg)));
    return o;
  }
  static __device__ __forceinline__ f32x4 get(const type &o, int t, int, const float *, const float *) {
    return f32x4{bf2f(o.v[t][0]), bf2f(o.v[t][1]), bf2f(o.v[t][2]), bf2f(o.v[t][3])};
  }
};
template <int NV>
struct RawAct<float, NV, false> {
  struct type { f32x4 v[4]; };
  static __device__ __forceinline__ type load(int cell, int lg, const float *h, const float *) {
    type o;
#pragma unroll
    for (int t = 0; t < 4; t++) o.v[t] = load_f4(h + h_off(h, cell, lch(t, lg)));
    return o;
  }
  static __device__ __forceinline__ f32x4 get(const type &o, int t, int, const float *, const float *) {
    return o.v[t];
  }
};
template <typename HT, int NV>
struct RawAct<HT, NV, true> {
  struct type { float u[NV]; };
  static __device__ __forceinline__ type load(int cell, int, const HT *, const float *r) {
    type o;
#pragma unroll
    for (int k = 0; k < NV; k++) o.u[k] = r[(size_t)cell * NV + k];
    return o;
  }
  static __device__ __forceinline__ f32x4 get(const type &o, int t, int lg, const float *W_in,
                                              const float *inv_s) {
    f32x4 h;
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int ch = lch(t, lg) + q;
      float v = 0.f;
#pragma unroll
      for (int k = 0; k < NV; k++) v += W_in[ch * NV + k] * (o.u[k] * inv_s[k]);
      h[q] = v;
    }
    return h;
  }
};

// Edge blocks in tile order (what the forward layers read).  For tile t and
// direction d the entries of the 16 cells form one run of kEdgeRun<NV> BF16,
// groups g of 16 cells x 4 entries 4g .. 4g + 3: four groups for nv = 4
// (256 values), three for nv = 3 (192 values: entries 0-3, 4-7, and entry 8
// followed by three zeros).  Lane group lg of a wave takes entries
// 4 lg .. 4 lg + 3 of cell lr (the B operand of the edge gate) with one
// 8-byte load: each group of 16 lanes reads 128 contiguous bytes; entries
// past nv^2 are zero.  (Loading the ninth entry alone, 2 bytes per lane, in a
// second instruction is slower, and so is a run of exactly nv^2 entries per
// cell with the six ninth entries in one 12-byte load.)  Cells past n (last
// tile) hold zeros.
template <int NV>
constexpr int kEdgeRun = NV == 3 ? 192 : 256;

template <int NV>
__device__ __forceinline__ bf16x4 load_edge_tiled(const short *__restrict__ Et, int tile, int d, int lg,
                                                  int lr) {
  const short *run = Et + ((size_t)tile * kDir + d) * kEdgeRun<NV>;
  if constexpr (NV == 4) {
    return __builtin_nontemporal_load(reinterpret_cast<const bf16x4 *>(run + lg * 64 + lr * 4));
  } else {
    // lane group 3 reads group 2's values again: they meet the zero columns
    // (k >= nv^2) of the W_e operand.  No branch or select on the loaded
    // value, so no wait for it before its use
    return __builtin_nontemporal_load(reinterpret_cast<const bf16x4 *>(run + min(lg, 2) * 64 + lr * 4));
  }
}

// Workgroups of the layer kernel: enough to fill the chip several times over;
// each wave loops over tiles.
constexpr int kLayerMaxBlocks = 2048;
constexpr int kXcds = 8;  // accelerator complex dies of the MI355X, each with its own L2
constexpr int kWPad = kHid + 8;  // LDS row of W_s / W_m (BF16): padded, 16-byte aligned
constexpr int kColWaves = 4096;  // target wave count of the z-column schedule (4 per SIMD)

// One message-passing layer.  One wavefront per tile of 16 consecutive cells;
// lane l owns cell c0 + l % 16 and the hidden channels lch(t, l / 16) + q
// (t, q = 0..3).  The weights are the MFMA A operand and the activations the
// B operand, so every product comes out with cells along the lanes:
//   g^T = W_e e^T (per direction, 16x16x16),  a^T = W_s h^T + W_m m^T (16x16x32)
// and the messages m = sum_d g * h_nbr, accumulated in that layout, are
// directly the B operand of W_m.  Activations are read and written as four
// consecutive channels per lane (HT: FP32 rows, or BF16 in tile order, see
// h_off).  W_s and W_m
// are staged in LDS once per workgroup; W_e stays in registers.
// FIRST: the input activations h0 = W_in (r / s) are formed on the fly for the
//        cell and its neighbours (stored to h0_out when given).
// LAST:  the read-out (LrnOut) is written; h_out may then be null.
// m_out / a_out (optional) keep the messages and pre-activations for the
// backward pass.
// Per-workgroup set-up shared by both layer kernels: W_s and W_m staged in
// LDS, 1 / s_k, and this lane's slice of W_e with the edge scaling folded in:
// (W_e S^{-1} e S)_j = sum_k W_e[j][k] f_k e_k, f_k = s_c / s_r for k = r NV + c,
// so the stored edge blocks are the B operand as they are.
// The matrix-core A operands of one lane (lane l = 16 lg + lr of a wave),
// the same in every wave of the workgroup, formed once per workgroup in LDS;
// we and win (used six times per tile) are then held in registers, wout (used
// once per tile) is read from LDS where it is used:
//   we[t]    this lane's slice of W_e with the edge scaling folded in, rows in
//            the order of output tile t;
//   win[t]   rows of W_in in the order of output tile t (first layer: the A
//            operand of h0_nbr = W_in (u / s), depth nv padded to 16);
//   wout[ks] rows 0 .. nv-1 of W_out, channels 32 ks .. 32 ks + 31 (last layer:
//            the A operand of the read-out W_out h3, rows nv .. 15 zero).
// Unused operands are zero.
template <int NV>
struct LaneOps {
  bf16x4 we[4];
  bf16x4 win[4];
  bf16x8 wout[2];
};

// Per-workgroup set-up shared by both layer kernels: W_s and W_m staged in
// LDS, the bias, the lane operands above, and 1 / s_k in registers.  The edge
// scaling (W_e S^{-1} e S)_j = sum_k W_e[j][k] f_k e_k, f_k = s_c / s_r for
// k = r NV + c, is folded into we, so the stored edge blocks are the B operand
// as they are.  The tile loops read the LDS copies through an offset the
// compiler cannot see through, so that these loop-invariant values are not
// held in registers for the whole loop.
template <int NV, bool FIRST, bool LAST>
__device__ __forceinline__ void layer_setup(short (&Wl)[2][kHid][kWPad], float (&bias_s)[kHid],
                                            LaneOps<NV> (&ops)[64], const short *__restrict__ W_s,
                                            const short *__restrict__ W_m, const float *__restrict__ W_e,
                                            const float *__restrict__ bias, const float *__restrict__ W_in,
                                            const float *__restrict__ W_out, const float *__restrict__ s_ptr,
                                            float (&inv_s)[NV], LaneOps<NV> &mine) {
  for (int v = threadIdx.x; v < 2 * kHid * kHid / 4; v += kBlock) {
    const int mtx = v / (kHid * kHid / 4), e = (v % (kHid * kHid / 4)) * 4;
    const short *src = (mtx == 0 ? W_s : W_m) + e;
    *reinterpret_cast<bf16x4 *>(&Wl[mtx][e / kHid][e % kHid]) = load_bf4(src);
  }
  for (int v = threadIdx.x; v < kHid; v += kBlock) bias_s[v] = bias[v];
  if (threadIdx.x < 64) {
    const int lr = threadIdx.x & 15, lg = threadIdx.x >> 4;
    LaneOps<NV> o;
#pragma unroll
    for (int t = 0; t < 4; t++)
#pragma unroll
      for (int q = 0; q < 4; q++) {
        // row lr of output tile t is channel lch(t, lr / 4) + lr % 4
        const int k = 4 * lg + q, row = lch(t, lr >> 2) + (lr & 3);
        o.we[t][q] = k < NV * NV ? f2bf(W_e[row * NV * NV + k] * edge_factor<NV>(k, s_ptr)) : short(0);
        o.win[t][q] = FIRST && k < NV ? f2bf(W_in[row * NV + k]) : short(0);
      }
#pragma unroll
    for (int ks = 0; ks < 2; ks++)
#pragma unroll
      for (int j = 0; j < 8; j++)
        o.wout[ks][j] = LAST && lr < NV ? f2bf(W_out[lr * kHid + 32 * ks + 8 * lg + j]) : short(0);
    ops[threadIdx.x] = o;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < NV; k++) {
    const float sk = s_ptr[k];
    inv_s[k] = sk > 0.f ? 1.f / sk : 0.f;
  }
  const LaneOps<NV> &o = ops[threadIdx.x & 63];
#pragma unroll
  for (int t = 0; t < 4; t++) {
    mine.we[t] = o.we[t];
    mine.win[t] = o.win[t];
  }
}

// A tile's own activations as layer_tile reads them: four FP32 quads (the
// first layer's h0, FP32 activations), or the BF16 row itself, widened where
// it is used.  BF16 -> FP32 -> BF16 is exact, so the BF16 operand of W_s is
// the row as loaded; keeping only the row spares the 16 registers of a
// widened copy in the inference layers.
struct OwnF32 {
  f32x4 v[4];
  __device__ __forceinline__ f32x4 get(int t) const { return v[t]; }
  __device__ __forceinline__ bf16x8 pair(int ks) const {
    return cat8(cvt4(v[2 * ks][0], v[2 * ks][1], v[2 * ks][2], v[2 * ks][3]),
                cvt4(v[2 * ks + 1][0], v[2 * ks + 1][1], v[2 * ks + 1][2], v[2 * ks + 1][3]));
  }
};
struct OwnBF16 {
  bf16x4 v[4];
  __device__ __forceinline__ f32x4 get(int t) const {
    return f32x4{bf2f(v[t][0]), bf2f(v[t][1]), bf2f(v[t][2]), bf2f(v[t][3])};
  }
  __device__ __forceinline__ bf16x8 pair(int ks) const { return cat8(v[2 * ks], v[2 * ks + 1]); }
};

// The arithmetic of one tile, shared by both layer kernels: given the cell's
// activations hv, the raw activations of its six neighbours (direction d =
// -x, +x, -y, +y, -z, +z; for an absent neighbour any finite row, its edge
// block being zero) and the six edge blocks, form the messages, the K = 32
// products, the update and the stores.  Lanes with ok == false store nothing.
template <int NV, bool FIRST, bool LAST, typename HT, typename ZT, typename XT, typename OWN>
__device__ __forceinline__ void layer_tile(int cell, bool ok, int lr, int lg, const OWN &hv,
                                           const typename RawAct<HT, NV, FIRST>::type (&raw)[kDir],
                                           const bf16x4 (&rawe)[kDir], const LaneOps<NV> &ops,
                                           const LaneOps<NV> &ops_lds,
                                           const short (&Wl)[2][kHid][kWPad], const float *__restrict__ W_in,
                                           const float (&inv_s)[NV], const float *__restrict__ bias,
                                           const float *__restrict__ r, const float *__restrict__ s_ptr,
                                           HT *__restrict__ hout, float *__restrict__ h0_out,
                                           float *__restrict__ m_out, float *__restrict__ a_out,
                                           const LrnOut<ZT, XT> &out, ZT *__restrict__ zout) {
  // the last layer's output terms of component k = lg of the cell (r_k, s_k
  // and x1's p or T part), loaded before the matrix work so that their
  // latency overlaps it
  float rpre = 0.f, spre = 0.f, xpre = 0.f;
  if constexpr (LAST) {
    if (ok && lg < NV) {
      rpre = r[(size_t)cell * NV + lg];
      spre = s_ptr[lg];
      if (!out.z2_out && out.dp && lg == out.ip) xpre = float(out.dp[cell]);
      if (!out.z2_out && out.dT && lg == out.iT) xpre = float(out.dT[cell]);
    }
  }
  __builtin_amdgcn_sched_barrier(0);
  f32x4 macc[4];
#pragma unroll
  for (int t = 0; t < 4; t++) macc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int d = 0; d < kDir; d++) {
    if constexpr (FIRST) {
      // the neighbour's h0 = W_in (u / s) on the matrix cores: B operand
      // rows k < nv hold u_k / s_k of the neighbour of cell lr (lane group 0)
      bf16x4 ub = {0, 0, 0, 0};
#pragma unroll
      for (int k = 0; k < NV; k++) ub[k] = lg == 0 ? f2bf(raw[d].u[k] * inv_s[k]) : short(0);
#pragma unroll
      for (int t = 0; t < 4; t++) {
        const f32x4 g = mfma16(ops.we[t], rawe[d], f32x4{0.f, 0.f, 0.f, 0.f});
        macc[t] += g * mfma16(ops.win[t], ub, f32x4{0.f, 0.f, 0.f, 0.f});
      }
      // one direction at a time: keeps the products of the next direction
      // from being hoisted (register pressure)
      __builtin_amdgcn_sched_barrier(0);
    } else {
#pragma unroll
      for (int t = 0; t < 4; t++) {
        const f32x4 g = mfma16(ops.we[t], rawe[d], f32x4{0.f, 0.f, 0.f, 0.f});
        macc[t] += g * RawAct<HT, NV, FIRST>::get(raw[d], t, lg, W_in, inv_s);
      }
    }
  }
  __builtin_amdgcn_sched_barrier(0);
  f32x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; t++) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int ks = 0; ks < 2; ks++) {
    // B operands: channels 32 ks + 8 lg .. + 7 = slots 2 ks, 2 ks + 1
    const bf16x8 hb = hv.pair(ks);
    const bf16x8 mb = cat8(cvt4(macc[2 * ks][0], macc[2 * ks][1], macc[2 * ks][2], macc[2 * ks][3]),
                           cvt4(macc[2 * ks + 1][0], macc[2 * ks + 1][1], macc[2 * ks + 1][2], macc[2 * ks + 1][3]));
#pragma unroll
    for (int t = 0; t < 4; t++) {
      const int row = lch(t, lr >> 2) + (lr & 3);
      const bf16x8 ws = *reinterpret_cast<const bf16x8 *>(&Wl[0][row][32 * ks + 8 * lg]);
      const bf16x8 wm = *reinterpret_cast<const bf16x8 *>(&Wl[1][row][32 * ks + 8 * lg]);
      acc[t] = mfma32(ws, hb, acc[t]);
      acc[t] = mfma32(wm, mb, acc[t]);
    }
  }
  f32x4 hnew[4];
#pragma unroll
  for (int t = 0; t < 4; t++) {
    f32x4 a;
#pragma unroll
    for (int q = 0; q < 4; q++) {
      a[q] = acc[t][q] + bias[lch(t, lg) + q];
      hnew[t][q] = hv.get(t)[q] + fmaxf(a[q], 0.f);
    }
    if (ok) {
      const size_t o = (size_t)cell * kHid + lch(t, lg);
      if (hout) store_h4(hout + h_off(hout, cell, lch(t, lg)), hnew[t]);
      if (m_out) store_f4(m_out + o, macc[t]);
      if (a_out) store_f4(a_out + o, a);
      if (FIRST && h0_out) store_f4(h0_out + o, hv.get(t));
    }
  }
  if constexpr (LAST) {
    // read-out (W_out h3)_k on the matrix cores: D row k, column lr lands in
    // lane (lr, k / 4), register k % 4; lane group 0 holds the nv <= 4 values
    f32x4 ro = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 2; ks++) {
      const bf16x8 hb = cat8(cvt4(hnew[2 * ks][0], hnew[2 * ks][1], hnew[2 * ks][2], hnew[2 * ks][3]),
                             cvt4(hnew[2 * ks + 1][0], hnew[2 * ks + 1][1], hnew[2 * ks + 1][2],
                                  hnew[2 * ks + 1][3]));
      ro = mfma32(ops_lds.wout[ks], hb, ro);
    }
    // component k of column lr moves to lane (lr, k): the lanes of a tile
    // then store nv consecutive values per cell
    float rk = 0.f;
#pragma unroll
    for (int k = 0; k < NV; k++) {
      const float v = __shfl(ro[k], lr, 64);
      if (lg == k) rk = v;
    }
    if (ok && lg < NV) {
      const size_t t = (size_t)cell * NV + lg;
      float z = rpre + spre * rk;
      if (out.z2_out) {
        out.z2_out[t] = z;
      } else {
        if ((out.dp && lg == out.ip) || (out.dT && lg == out.iT)) z += xpre;
        zout[t] = ZT(z);
      }
    }
  }
}

// One message-passing layer over tiles in cell order.  Any 7-point cell graph
// (neighbours by presence mask and the three axis strides).
template <int NV, bool FIRST, bool LAST, typename HT, typename ZT, typename XT>
__device__ __forceinline__ void lrn_layer_tiles(
    int n, const unsigned char *__restrict__ nmask, int3 stride, const short *__restrict__ Et,
    const float *__restrict__ s_ptr, const HT *__restrict__ hin, const float *__restrict__ r, const float *__restrict__ W_in,
    const float *__restrict__ W_e, const short *__restrict__ W_s, const short *__restrict__ W_m,
    const float *__restrict__ bias, HT *__restrict__ hout, float *__restrict__ h0_out,
    float *__restrict__ m_out, float *__restrict__ a_out, const LrnOut<ZT, XT> &out) {
  __shared__ __attribute__((aligned(16))) short Wl[2][kHid][kWPad];
  // first layer: W_in in LDS for the cell's own h0 (read in the tile loop,
  // not held in registers)
  __shared__ float Win_s[FIRST ? kHid * NV : 1];
  __shared__ float bias_s[kHid];
  __shared__ LaneOps<NV> ops_s[64];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int lr = l & 15, lg = l >> 4;
  const int ntiles = (n + 15) / 16;
  if constexpr (FIRST)
    for (int v = threadIdx.x; v < kHid * NV; v += kBlock) Win_s[v] = W_in[v];
  float inv_s[NV];
  LaneOps<NV> ops;
  // (its barrier covers Win_s)
  layer_setup<NV, FIRST, LAST>(Wl, bias_s, ops_s, W_s, W_m, W_e, bias, W_in, out.W_out, s_ptr, inv_s, ops);
  ZT *const zout = lrn_zout<LAST>(out);
  using Raw = RawAct<HT, NV, FIRST>;
  const int off[kDir] = {-stride.x, stride.x, -stride.y, stride.y, -stride.z, stride.z};
  // XCD-aware order: workgroups are dealt to the 8 XCDs round robin, so the
  // workgroups of one XCD (blockIdx % 8) take one contiguous eighth of the
  // tiles, in increasing order; a tile's neighbours along the slower axes were
  // then fetched recently into the same XCD's L2.  (gridDim.x is a multiple of 8.)
  const int nwx = (gridDim.x / kXcds) * (kBlock / 64);         // waves per XCD
  const int per = (ntiles + kXcds - 1) / kXcds;                // tiles per XCD
  const int xcd = blockIdx.x % kXcds;
  const int t_end = min(ntiles, (xcd + 1) * per);
  const int tile0 = xcd * per + (blockIdx.x / kXcds) * (kBlock / 64) + w;
  // presence mask of the next tile, loaded one iteration ahead
  unsigned mk_next = tile0 < t_end ? nmask[min(tile0 * 16 + lr, n - 1)] : 0u;
  for (int tile = tile0; tile < t_end; tile += nwx) {
    const int cell = tile * 16 + lr;
    const bool ok = cell < n;
    // lanes past the end read the last cell; their results are never stored
    const int cl = ok ? cell : n - 1;
    const unsigned mk = mk_next;  // bit d: neighbour cell + off[d] exists
    if (tile + nwx < t_end) mk_next = nmask[min((tile + nwx) * 16 + lr, n - 1)];
    // all loads are issued first and consumed direction by direction.  An
    // absent neighbour has a zero edge block, so its (any finite) activations
    // -- the cell's own are read in its place -- add zero.
    const typename Raw::type own = Raw::load(cl, lg, hin, r);
    typename Raw::type raw[kDir];
    bf16x4 rawe[kDir];
#pragma unroll
    for (int d = 0; d < kDir; d++) {
      rawe[d] = load_edge_tiled<NV>(Et, tile, d, lg, lr);
      raw[d] = Raw::load((mk >> d) & 1u ? cl + off[d] : cl, lg, hin, r);
    }
    // an offset the compiler cannot see through keeps the LDS reads of W_in,
    // the bias and the lane operands in the loop
    int z0 = 0;
    asm volatile("" : "+v"(z0));
    OwnF32 hv;
#pragma unroll
    for (int t = 0; t < 4; t++) hv.v[t] = Raw::get(own, t, lg, FIRST ? Win_s + z0 : W_in, inv_s);
    layer_tile<NV, FIRST, LAST, HT, ZT, XT>(cell, ok, lr, lg, hv, raw, rawe, ops, ops_s[l + z0], Wl, W_in,
                                           inv_s, bias_s + z0, r, s_ptr, hout, h0_out, m_out, a_out, out, zout);
  }
}

#define CPTR_LRN_LAYER_ARGS                                                                                 \
  int n, const unsigned char *__restrict__ nmask, int3 stride, const short *__restrict__ Et,              \
      const float *__restrict__ s_ptr, const HT *__restrict__ hin, const float *__restrict__ r,           \
      const float *__restrict__ W_in, const float *__restrict__ W_e, const short *__restrict__ W_s,       \
      const short *__restrict__ W_m, const float *__restrict__ bias, HT *__restrict__ hout,                \
      float *__restrict__ h0_out, float *__restrict__ m_out, float *__restrict__ a_out, LrnOut<ZT, XT> out
#define CPTR_LRN_LAYER_CALL \
  lrn_layer_tiles<NV, FIRST, LAST, HT, ZT, XT>(n, nmask, stride, Et, s_ptr, hin, r, W_in, W_e, W_s, W_m, bias, hout, \
                                              h0_out, m_out, a_out, out)

template <int NV, bool FIRST, bool LAST, typename HT, typename ZT, typename XT>
__global__ void __launch_bounds__(kBlock) k_lrn_layer(CPTR_LRN_LAYER_ARGS) {
  CPTR_LRN_LAYER_CALL;
}

// the same for the first layer of the forward pass, whose h0 = W_in (r / s)
// of seven cells per tile needs many registers: held to three waves per SIMD
template <int NV, bool FIRST, bool LAST, typename HT, typename ZT, typename XT>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3)))
k_lrn_layer_first(CPTR_LRN_LAYER_ARGS) {
  CPTR_LRN_LAYER_CALL;
}
#undef CPTR_LRN_LAYER_CALL
#undef CPTR_LRN_LAYER_ARGS

// x-neighbour rows by lane shuffle: lane lr of each 16-lane DPP row takes the
// value of lane lr - 1 (row_shr:1) or lr + 1 (row_shl:1); the lane at the end
// of the row, which has no such lane, keeps `edge` (bound_ctrl off).
template <typename R, int CTRL>
__device__ __forceinline__ R shuffle_row(const R &own, const R &edge) {
  static_assert(sizeof(R) % 4 == 0, "raw activations are whole dwords");
  constexpr int nd = sizeof(R) / 4;
  struct D { int v[nd]; };
  const D o = __builtin_bit_cast(D, own), e = __builtin_bit_cast(D, edge);
  D res;
#pragma unroll
  for (int i = 0; i < nd; i++) res.v[i] = __builtin_amdgcn_update_dpp(e.v[i], o.v[i], CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(R, res);
}
constexpr int kDppRowShr1 = 0x111;  // lane i <- lane i - 1 within a row of 16
constexpr int kDppRowShl1 = 0x101;  // lane i <- lane i + 1 within a row of 16

// The same layer on a structured grid whose cells are numbered x fastest with
// a plane (stride.z) of P whole tiles: a wave walks a column of tiles along z
// (tile (p, z) = cells (z P + p) 16 ..), so the -z row is the previous tile's
// own and the +z row the next tile's own, kept in registers; -x and +x come
// from the lanes next door, with one load for the two lanes at the tile ends;
// only +-y are gathered.  Columns are cut into chunks of zlen planes; each
// XCD takes a contiguous range of columns (with all their chunks), so the
// waves that share +-y rows run on the same L2 at the same time.  The result
// is the one of k_lrn_layer, bit for bit: every neighbour row that is present
// is the same row, every absent one finite (and multiplied by zero).
template <int NV, bool FIRST, bool LAST, typename HT, typename ZT, typename XT>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) k_lrn_layer_col(
    int n, int P, int nz, int zlen, int sy, const short *__restrict__ Et, const float *__restrict__ s_ptr,
    const HT *__restrict__ hin, const float *__restrict__ r, const float *__restrict__ W_in,
    const float *__restrict__ W_e, const short *__restrict__ W_s, const short *__restrict__ W_m,
    const float *__restrict__ bias, HT *__restrict__ hout, LrnOut<ZT, XT> out) {
  __shared__ __attribute__((aligned(16))) short Wl[2][kHid][kWPad];
  __shared__ float bias_s[kHid];
  __shared__ LaneOps<NV> ops_s[64];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int lr = l & 15, lg = l >> 4;
  float inv_s[NV];
  LaneOps<NV> ops;
  layer_setup<NV, FIRST, LAST>(Wl, bias_s, ops_s, W_s, W_m, W_e, bias, W_in, out.W_out, s_ptr, inv_s, ops);
  ZT *const zout = lrn_zout<LAST>(out);
  using Raw = RawAct<HT, NV, FIRST>;
  using RT = typename Raw::type;
  const int sz = P * 16;
  const int nchunk = (nz + zlen - 1) / zlen;
  const int items = P * nchunk;                       // (column, chunk) pairs
  const int per = (items + kXcds - 1) / kXcds;        // per XCD, column-major
  const int nwx = (gridDim.x / kXcds) * (kBlock / 64);
  const int xcd = blockIdx.x % kXcds;
  const int i_end = min(items, (xcd + 1) * per);
  for (int item = xcd * per + (blockIdx.x / kXcds) * (kBlock / 64) + w; item < i_end; item += nwx) {
    const int p = item / nchunk, z0 = (item % nchunk) * zlen, z1 = min(nz, z0 + zlen);
    int cell = (z0 * P + p) * 16 + lr;
    RT rp = Raw::load(z0 > 0 ? cell - sz : cell, lg, hin, r);
    RT rc = Raw::load(cell, lg, hin, r);
    for (int z = z0; z < z1; z++, cell += sz) {
      const RT rn = Raw::load(z + 1 < nz ? cell + sz : cell, lg, hin, r);
      RT raw[kDir];
      raw[2] = Raw::load(max(cell - sy, 0), lg, hin, r);
      raw[3] = Raw::load(min(cell + sy, n - 1), lg, hin, r);
      RT xe = rc;
      if (lr == 0 || lr == 15) xe = Raw::load(lr == 0 ? max(cell - 1, 0) : min(cell + 1, n - 1), lg, hin, r);
      bf16x4 rawe[kDir];
#pragma unroll
      for (int d = 0; d < kDir; d++)
        rawe[d] = load_edge_tiled<NV>(Et, cell >> 4, d, lg, lr);
      raw[0] = shuffle_row<RT, kDppRowShr1>(rc, xe);
      raw[1] = shuffle_row<RT, kDppRowShl1>(rc, xe);
      raw[4] = rp;
      raw[5] = rn;
      int z0 = 0;  // keeps the LDS reads of the bias and the lane operands in the loop
      asm volatile("" : "+v"(z0));
      if constexpr (!FIRST && std::is_same_v<HT, short>) {
        const OwnBF16 hv{{rc.v[0], rc.v[1], rc.v[2], rc.v[3]}};
        layer_tile<NV, FIRST, LAST, HT, ZT, XT>(cell, true, lr, lg, hv, raw, rawe, ops, ops_s[l + z0], Wl, W_in,
                                               inv_s, bias_s + z0, r, s_ptr, hout, nullptr, nullptr, nullptr, out,
                                               zout);
      } else {
        OwnF32 hv;
#pragma unroll
        for (int t = 0; t < 4; t++) hv.v[t] = Raw::get(rc, t, lg, W_in, inv_s);
        layer_tile<NV, FIRST, LAST, HT, ZT, XT>(cell, true, lr, lg, hv, raw, rawe, ops, ops_s[l + z0], Wl, W_in,
                                               inv_s, bias_s + z0, r, s_ptr, hout, nullptr, nullptr, nullptr, out,
                                               zout);
      }
      rp = rc;
      rc = rn;
    }
  }
}

// ---------------------------------------------------------------------------
// training
// ---------------------------------------------------------------------------
// y = A^T x for FP64 BSR with a structurally symmetric pattern; tpos[k] is the
// position of block (j, i) for the block (i, j) stored at k.  One thread per
// (block row, component).
template <int NV>
__global__ void __launch_bounds__(kBlock) k_bsr_spmv_t(int n, const int *__restrict__ rp,
                                                       const int *__restrict__ ci,
                                                       const int *__restrict__ tpos,
                                                       const double *__restrict__ vals,
                                                       const double *__restrict__ x,
                                                       double *__restrict__ y) {
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const int j = t / NV, c = t - j * NV;
  if (j >= n) return;
  double acc = 0.0;
  for (int k = rp[j]; k < rp[j + 1]; k++) {
    const int i = ci[k];
    const double *blk = vals + (size_t)tpos[k] * NV * NV;  // block (i, j)
#pragma unroll
    for (int r = 0; r < NV; r++) acc += blk[r * NV + c] * x[(size_t)i * NV + r];
  }
  y[t] = acc;
}

// dout = s * scale * dz;  dh3 = W_out^T dout;  partial dW_out (per workgroup)
template <int NV>
__global__ void __launch_bounds__(kBlock) k_lrn_out_bwd(int n, const double *__restrict__ dz,
                                                        double scale, const float *__restrict__ s_ptr,
                                                        const float *__restrict__ W_out,
                                                        const float *__restrict__ h3,
                                                        float *__restrict__ dh3,
                                                        float *__restrict__ part) {
  // thread = (cell, hidden unit); partial dW_out[k][c] over the cells of the block
  __shared__ float red[kBlock / kHid][NV][kHid];
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const int i = t / kHid, c = t % kHid;
  float dout[NV];
  float acc = 0.f;
  const bool live = i < n;
#pragma unroll
  for (int k = 0; k < NV; k++) {
    dout[k] = live ? float(scale * dz[(size_t)i * NV + k]) * s_ptr[k] : 0.f;
    acc += W_out[k * kHid + c] * dout[k];
  }
  const float hv = live ? h3[(size_t)i * kHid + c] : 0.f;
  if (live) dh3[(size_t)i * kHid + c] = acc;
  const int slot = threadIdx.x / kHid;
#pragma unroll
  for (int k = 0; k < NV; k++) red[slot][k][c] = dout[k] * hv;
  __syncthreads();
  if (threadIdx.x < kHid) {
#pragma unroll
    for (int k = 0; k < NV; k++) {
      float sum = 0.f;
      for (int q = 0; q < kBlock / kHid; q++) sum += red[q][k][threadIdx.x];
      part[(size_t)blockIdx.x * NV * kHid + k * kHid + threadIdx.x] = sum;
    }
  }
}

// Per layer, first backward pass (one wave per 16-cell tile, grid-stride):
//   da = dh * [a > 0];  dm = da W_m;  dh_own = dh + da W_s
//   dW_s += da^T h, dW_m += da^T m, db += sum da, dW_e += sum_d (dm * h_nbr)^T E_d
// The weight-gradient partials of every wave go to `part` (reduced later in a
// fixed order).  W_sT / W_mT are the transposes in BF16.
template <int NV>
__global__ void __launch_bounds__(kBlock) k_lrn_layer_bwd1(
    int n, int ntiles, const int *__restrict__ nbr, const short *__restrict__ E,
    const float *__restrict__ s_ptr,
    const float *__restrict__ hprev, const float *__restrict__ m, const float *__restrict__ a,
    const float *__restrict__ dh, const short *__restrict__ W_sT, const short *__restrict__ W_mT,
    float *__restrict__ dm_out, float *__restrict__ dh_own, float *__restrict__ part) {
  __shared__ float sda[kBlock / 64][16][kHid + 4];
  __shared__ float sdm[kBlock / 64][16][kHid + 4];
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int lr = l & 15, lg = l >> 4;
  f32x4 gWs[4][4], gWm[4][4], gWe[4];
  float gb[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int x = 0; x < 4; x++) {
    gWe[x] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int y = 0; y < 4; y++) gWs[x][y] = gWm[x][y] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  const int wave_id = blockIdx.x * (kBlock / 64) + w;
  // every wave of a workgroup runs the same number of iterations (the loop
  // holds workgroup barriers); tiles past the end are all-padding tiles
  for (int base = blockIdx.x * (kBlock / 64); base < ntiles; base += gridDim.x * (kBlock / 64)) {
    const int tile = base + w;
    const int c0 = tile * 16;
    const int ca = c0 + lr;
    // da in A layout (rows = cells) and into LDS
    f32x4 dmacc[4], dhacc[4];
#pragma unroll
    for (int t = 0; t < 4; t++) dmacc[t] = dhacc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < 4; ks++) {
      const int k0 = 16 * ks + 4 * lg;
      float v[4] = {0.f, 0.f, 0.f, 0.f};
      if (ca < n) {
#pragma unroll
        for (int q = 0; q < 4; q++) {
          const size_t o = (size_t)ca * kHid + k0 + q;
          v[q] = a[o] > 0.f ? dh[o] : 0.f;
        }
      }
#pragma unroll
      for (int q = 0; q < 4; q++) sda[w][lr][k0 + q] = v[q];
      const bf16x4 dav = cvt4(v[0], v[1], v[2], v[3]);
#pragma unroll
      for (int t = 0; t < 4; t++) {
        dmacc[t] = mfma16(dav, load_bf4(W_mT + (lr + 16 * t) * kHid + k0), dmacc[t]);
        dhacc[t] = mfma16(dav, load_bf4(W_sT + (lr + 16 * t) * kHid + k0), dhacc[t]);
      }
    }
    // outputs in D layout; dm also into LDS
#pragma unroll
    for (int t = 0; t < 4; t++)
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const int cell = c0 + 4 * lg + q, col = lr + 16 * t;
        sdm[w][4 * lg + q][col] = dmacc[t][q];
        if (cell < n) {
          const size_t o = (size_t)cell * kHid + col;
          dm_out[o] = dmacc[t][q];
          dh_own[o] = dh[o] + dhacc[t][q];
        }
      }
    __syncthreads();
    // weight gradients, cells as the reduction dimension:
    //   A[c][cell] = da[cell][c] (lane: c = lr + 16 mt, cell = 4 lg + q)
    //   B[cell][k] = h[cell][k] or m[cell][k] (lane: cell = 4 lg + q, k = lr + 16 nt)
#pragma unroll
    for (int mt = 0; mt < 4; mt++) {
      const bf16x4 A = cvt4(sda[w][4 * lg + 0][lr + 16 * mt], sda[w][4 * lg + 1][lr + 16 * mt],
                            sda[w][4 * lg + 2][lr + 16 * mt], sda[w][4 * lg + 3][lr + 16 * mt]);
      gb[mt] += sda[w][4 * lg + 0][lr + 16 * mt] + sda[w][4 * lg + 1][lr + 16 * mt] +
                sda[w][4 * lg + 2][lr + 16 * mt] + sda[w][4 * lg + 3][lr + 16 * mt];
#pragma unroll
      for (int nt = 0; nt < 4; nt++) {
        float hb[4], mb[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
          const int cell = c0 + 4 * lg + q;
          const size_t o = (size_t)cell * kHid + lr + 16 * nt;
          hb[q] = cell < n ? hprev[o] : 0.f;
          mb[q] = cell < n ? m[o] : 0.f;
        }
        gWs[mt][nt] = mfma16(A, cvt4(hb[0], hb[1], hb[2], hb[3]), gWs[mt][nt]);
        gWm[mt][nt] = mfma16(A, cvt4(mb[0], mb[1], mb[2], mb[3]), gWm[mt][nt]);
      }
    }
    // dW_e[c][e] += sum_{cell,d} dm[cell][c] h[nbr(cell,d)][c] E[cell][d][e]
    for (int d = 0; d < kDir; d++) {
      int nb[4];
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const int cell = c0 + 4 * lg + q;
        nb[q] = cell < n ? nbr[(size_t)cell * kDir + d] : -1;
      }
      // B[cell][e] = E[cell][d][e]: lane cell = 4 lg + q, e = lr
      float eb[4];
      const float ef = edge_factor<NV>(lr, s_ptr);
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const int cell = c0 + 4 * lg + q;
        eb[q] = cell < n ? ef * __uint_as_float(uint32_t((unsigned short)E[((size_t)cell * kDir + d) * kEdge + lr]) << 16) : 0.f;
      }
      const bf16x4 B = cvt4(eb[0], eb[1], eb[2], eb[3]);
#pragma unroll
      for (int mt = 0; mt < 4; mt++) {
        float av[4];
#pragma unroll
        for (int q = 0; q < 4; q++)
          av[q] = nb[q] >= 0 ? sdm[w][4 * lg + q][lr + 16 * mt] * hprev[(size_t)nb[q] * kHid + lr + 16 * mt]
                             : 0.f;
        gWe[mt] = mfma16(cvt4(av[0], av[1], av[2], av[3]), B, gWe[mt]);
      }
    }
    __syncthreads();
  }
  // per-wave partials: [W_s 64x64 | W_m 64x64 | W_e 64x16 | b 64]
  constexpr int P = 2 * kHid * kHid + kHid * kEdge + kHid;
  float *out = part + (size_t)wave_id * P;
#pragma unroll
  for (int mt = 0; mt < 4; mt++)
#pragma unroll
    for (int nt = 0; nt < 4; nt++)
#pragma unroll
      for (int q = 0; q < 4; q++) {
        const int row = 16 * mt + 4 * lg + q, col = 16 * nt + lr;
        out[row * kHid + col] = gWs[mt][nt][q];
        out[kHid * kHid + row * kHid + col] = gWm[mt][nt][q];
      }
#pragma unroll
  for (int mt = 0; mt < 4; mt++)
#pragma unroll
    for (int q = 0; q < 4; q++) out[2 * kHid * kHid + (16 * mt + 4 * lg + q) * kEdge + lr] = gWe[mt][q];
  // db: lanes with the same lr hold partial sums of column lr + 16 mt over their 4 cells
#pragma unroll
  for (int mt = 0; mt < 4; mt++) {
    float v = gb[mt];
    v += __shfl_xor(v, 16, 64);
    v += __shfl_xor(v, 32, 64);
    if (lg == 0) out[2 * kHid * kHid + kHid * kEdge + lr + 16 * mt] = v;
  }
}

// Per layer, second backward pass: dh_prev_j = dh_own_j + sum over the
// neighbours i of j, with j = nbr(i, d), of dm_i * (W_e e_{i,d}).
// nbr_opp(j, d) = i with nbr(i, d) = j (the neighbour in the opposite direction).
template <int NV>
__global__ void __launch_bounds__(kBlock) k_lrn_layer_bwd2(int n, const int *__restrict__ nbr,
                                                           const short *__restrict__ E,
                                                           const float *__restrict__ s_ptr,
                                                           const short *__restrict__ W_e16,
                                                           const float *__restrict__ dm,
                                                           const float *__restrict__ dh_own,
                                                           float *__restrict__ dh_prev) {
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int lr = l & 15, lg = l >> 4;
  const int c0 = (blockIdx.x * (kBlock / 64) + w) * 16;
  f32x4 acc[4];
#pragma unroll
  for (int t = 0; t < 4; t++) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  for (int d = 0; d < kDir; d++) {
    const int od = d ^ 1;  // opposite direction
    // A row (lane lr): edge features of i = nbr(cell, od) in direction d
    const int cell_a = c0 + lr;
    const int ia = cell_a < n ? nbr[(size_t)cell_a * kDir + od] : -1;
    bf16x4 ea = bf16x4{0, 0, 0, 0};
    if (ia >= 0) ea = scale_edge4<NV>(load_bf4(E + ((size_t)ia * kDir + d) * kEdge + 4 * lg), 4 * lg, s_ptr);
    int ib[4];
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int cell = c0 + 4 * lg + q;
      ib[q] = cell < n ? nbr[(size_t)cell * kDir + od] : -1;
    }
#pragma unroll
    for (int t = 0; t < 4; t++) {
      const f32x4 g = mfma16(ea, load_bf4(W_e16 + (lr + 16 * t) * kEdge + 4 * lg), f32x4{0.f, 0.f, 0.f, 0.f});
#pragma unroll
      for (int q = 0; q < 4; q++)
        if (ib[q] >= 0) acc[t][q] += g[q] * dm[(size_t)ib[q] * kHid + lr + 16 * t];
    }
  }
#pragma unroll
  for (int t = 0; t < 4; t++)
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int cell = c0 + 4 * lg + q;
      if (cell >= n) continue;
      const size_t o = (size_t)cell * kHid + lr + 16 * t;
      dh_prev[o] = dh_own[o] + acc[t][q];
    }
}

// partial dW_in[c][k] = sum_cells dh0[cell][c] * r[cell][k] / s_k (per workgroup)
template <int NV>
__global__ void __launch_bounds__(kBlock) k_lrn_in_bwd(int n, const float *__restrict__ dh0,
                                                       const float *__restrict__ r,
                                                       const float *__restrict__ s_ptr,
                                                       float *__restrict__ part) {
  __shared__ float red[kBlock / kHid][kHid][NV];
  const int t = blockIdx.x * kBlock + threadIdx.x;
  const int i = t / kHid, c = t % kHid;
  const int slot = threadIdx.x / kHid;
  const float g = i < n ? dh0[(size_t)i * kHid + c] : 0.f;
#pragma unroll
  for (int k = 0; k < NV; k++) {
    const float s = s_ptr[k];
    const float inv = s > 0.f ? 1.f / s : 0.f;
    red[slot][c][k] = i < n ? g * (r[(size_t)i * NV + k] * inv) : 0.f;
  }
  __syncthreads();
  if (threadIdx.x < kHid) {
#pragma unroll
    for (int k = 0; k < NV; k++) {
      float sum = 0.f;
      for (int q = 0; q < kBlock / kHid; q++) sum += red[q][threadIdx.x][k];
      part[(size_t)blockIdx.x * kHid * NV + threadIdx.x * NV + k] = sum;
    }
  }
}

// out[e] (+)= sum_p part[p][e] in two passes with a fixed order: workgroup b
// sums the rows p = b, b + G, ... (coalesced along e) into mid[b][e]; then
// one thread per e sums mid[0..G-1][e].
constexpr int kSumGroups = 256;
__global__ void __launch_bounds__(kBlock) k_sum_partials_rows(const float *__restrict__ part, int np, int len,
                                                              float *__restrict__ mid) {
  for (int e = threadIdx.x; e < len; e += kBlock) {
    float s = 0.f;
    for (int p = blockIdx.x; p < np; p += gridDim.x) s += part[(size_t)p * len + e];
    mid[(size_t)blockIdx.x * len + e] = s;
  }
}
__global__ void __launch_bounds__(kBlock) k_sum_partials_cols(const float *__restrict__ mid, int groups, int len,
                                                              float *__restrict__ out, int accumulate) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= len) return;
  float s = 0.f;
  for (int b = 0; b < groups; b++) s += mid[(size_t)b * len + e];
  out[e] = accumulate ? out[e] + s : s;
}

// Adam step on the FP32 master weights (gradient already averaged)
__global__ void __launch_bounds__(kBlock) k_adam(int np, float *__restrict__ theta,
                                                 const float *__restrict__ grad,
                                                 float *__restrict__ m, float *__restrict__ v,
                                                 float lr, float b1, float b2, float eps,
                                                 float c1, float c2) {
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= np) return;
  const float g = grad[e];
  const float mm = b1 * m[e] + (1.f - b1) * g;
  const float vv = b2 * v[e] + (1.f - b2) * g * g;
  m[e] = mm;
  v[e] = vv;
  theta[e] -= lr * (mm / c1) / (sqrtf(vv / c2) + eps);
}

// BF16 operands from the FP32 master weights: per layer W_e (64 x 16, padded),
// W_s, W_m and their transposes.
template <int NV>
__global__ void __launch_bounds__(kBlock) k_lrn_pack(const float *__restrict__ theta,
                                                     short *__restrict__ packed) {
  constexpr int NIN = kHid * NV;
  constexpr int NL = kHid * NV * NV + 2 * kHid * kHid + kHid;
  constexpr int PL = kHid * kEdge + 4 * kHid * kHid;  // packed floats per layer
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= 3 * PL) return;
  const int layer = e / PL, o = e % PL;
  const float *L = theta + NIN + layer * NL;
  float v;
  if (o < kHid * kEdge) {
    const int c = o / kEdge, k = o % kEdge;
    v = k < NV * NV ? L[c * NV * NV + k] : 0.f;
  } else {
    const int q = o - kHid * kEdge, which = q / (kHid * kHid), p = q % (kHid * kHid);
    const int row = p / kHid, col = p % kHid;
    const float *Ws = L + kHid * NV * NV, *Wm = Ws + kHid * kHid;
    switch (which) {
      case 0: v = Ws[row * kHid + col]; break;
      case 1: v = Wm[row * kHid + col]; break;
      case 2: v = Ws[col * kHid + row]; break;
      default: v = Wm[col * kHid + row]; break;
    }
  }
  packed[e] = f2bf(v);
}

// grad_layer[e] += sum over waves of the layer partials, mapped from the
// partial layout [W_s | W_m | W_e (64 x 16) | b] to the parameter layout
// [W_e (64 x nv^2) | W_s | W_m | b]
template <int NV>
__global__ void __launch_bounds__(kBlock) k_lrn_reduce_layer(const float *__restrict__ part, int nw,
                                                             float *__restrict__ grad) {
  // part: nw rows of [W_s | W_m | W_e (64 x 16) | b] partial sums
  constexpr int NE = kHid * NV * NV, P = 2 * kHid * kHid + kHid * kEdge + kHid;
  const int e = blockIdx.x * kBlock + threadIdx.x;
  if (e >= NE + 2 * kHid * kHid + kHid) return;
  int src;
  if (e < NE) src = 2 * kHid * kHid + (e / (NV * NV)) * kEdge + e % (NV * NV);
  else if (e < NE + 2 * kHid * kHid) src = e - NE;
  else src = 2 * kHid * kHid + kHid * kEdge + (e - NE - 2 * kHid * kHid);
  float s = 0.f;
  for (int w = 0; w < nw; w++) s += part[(size_t)w * P + src];
  grad[e] += s;
}

}  // namespace cptr
