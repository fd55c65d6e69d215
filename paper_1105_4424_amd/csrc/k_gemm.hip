// k_gemm.hip -- the DOT task whose tilers form a dense matrix product.
//
// C[m, n] = sum_k A(m, k) B(k, n), FP32 accumulation on the matrix cores:
//   * BF16 operands: v_mfma_f32_32x32x16_bf16 (products exact in FP32)
//   * FP32 operands: v_mfma_f32_32x32x2_f32
// The kernels want both operands with k contiguous ("A[m][k]", "Bt[n][k]"),
// except that the large-tile BF16 kernel also takes B stored [K][N] as it is
// and transposes its fragments on the way out of LDS (gfx950's
// ds_read_b64_tr_b16).  Any other operand whose tiler walks k along a
// strided axis is first transposed into the library workspace by an
// LDS-tiled transpose kernel.
//
// Tiling: 128 x 128 outputs per workgroup of 4 waves (2 x 2), 64 x 64 per
// wave as 2 x 2 MFMA tiles of 32 x 32; the k-loop stages 128-byte rows of
// both operands in LDS (row pitch 144 B: the 16-lane phases of ds_read_b128
// touch distinct banks), double-buffered, with the next tile prefetched into
// registers while the current one feeds the MFMAs.  Workgroup ids are
// remapped so that each XCD (ids are dealt round-robin to the 8 XCDs) works
// on a contiguous, grouped band of output tiles and shares A / B panels in
// its own L2.
#include <hip/hip_runtime.h>

#include <string>

#include "rsm_internal.h"

namespace rsm {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx16 __attribute__((ext_vector_type(16)));

constexpr int kBM = 128;
constexpr int kBN = 128;
constexpr int kRowBytes = 128;        // one LDS row = 128 bytes of k
constexpr int kPitch = 144;           // padded LDS row pitch in bytes
constexpr int kThreads = 256;
constexpr int kXcds = 8;
constexpr int kGroupM = 8;            // tile rows per raster group

template <typename T>
struct Mfma;

template <>
struct Mfma<uint16_t> {
  static constexpr int kPerChunk = 8;  // elements per 16-byte chunk
  __device__ static __forceinline__ floatx16 step(uint4 a, uint4 b, floatx16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8, a),
                                                   __builtin_bit_cast(bf16x8, b), c, 0, 0, 0);
  }
};

template <>
struct Mfma<float> {
  static constexpr int kPerChunk = 4;
  // k-slot h of instruction s holds physical k = 8g + 4h + s: the same
  // mapping on both operands, so the four products cover the 8 k values.
  __device__ static __forceinline__ floatx16 step(uint4 a, uint4 b, floatx16 c) {
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.x), __uint_as_float(b.x), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.y), __uint_as_float(b.y), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.z), __uint_as_float(b.z), c, 0, 0, 0);
    c = __builtin_amdgcn_mfma_f32_32x32x2f32(__uint_as_float(a.w), __uint_as_float(b.w), c, 0, 0, 0);
    return c;
  }
};

struct TnArgs {
  int32_t M, N, K;
  int64_t lda;   // elements between rows of A[m][k]
  int64_t ldb;   // elements between rows of Bt[n][k]
  int64_t ldc;
  const void* a;
  const void* b;
  float* c;
  int32_t tiles_m, tiles_n;
};

// Maps a hardware workgroup id to an output tile: XCD-contiguous bands,
// grouped raster inside each band.
__device__ __forceinline__ void tile_of(int bid, int tiles_m, int tiles_n, int* tm, int* tn) {
  const int total = tiles_m * tiles_n;
  int logical = bid;
  if (total % kXcds == 0) logical = (bid % kXcds) * (total / kXcds) + bid / kXcds;
  const int per_group = kGroupM * tiles_n;
  const int group = logical / per_group;
  const int first_m = group * kGroupM;
  const int gm = (tiles_m - first_m) < kGroupM ? (tiles_m - first_m) : kGroupM;
  const int in_group = logical - group * per_group;
  *tm = first_m + in_group % gm;
  *tn = in_group / gm;
}

template <typename T>
__global__ void __launch_bounds__(kThreads, 2) gemm_tn_kernel(TnArgs p) {
  constexpr int E = Mfma<T>::kPerChunk;      // elements per 16-byte chunk
  constexpr int BK = kRowBytes / sizeof(T);  // k elements per LDS row
  __shared__ __attribute__((aligned(16))) unsigned char lds[2][2][kBM * kPitch];

  int tm, tn;
  tile_of(blockIdx.x, p.tiles_m, p.tiles_n, &tm, &tn);
  const int m0 = tm * kBM, n0 = tn * kBN;
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int li = lane & 31, lh = lane >> 5;

  const T* A = static_cast<const T*>(p.a);
  const T* B = static_cast<const T*>(p.b);

  // global -> register staging: 4 chunks of A and 4 of B per thread
  uint4 ra[4], rb[4];
#define RSM_GEMM_LOAD(K0)                                                                  \
  _Pragma("unroll") for (int j = 0; j < 4; ++j) {                                          \
    const int q = t + kThreads * j;                                                        \
    const int row = q >> 3, kk = (K0) + (q & 7) * E;                                       \
    const int am = m0 + row, bn = n0 + row;                                                \
    ra[j] = (am < p.M && kk < p.K) ? *reinterpret_cast<const uint4*>(A + am * p.lda + kk)  \
                                   : make_uint4(0, 0, 0, 0);                               \
    rb[j] = (bn < p.N && kk < p.K) ? *reinterpret_cast<const uint4*>(B + bn * p.ldb + kk)  \
                                   : make_uint4(0, 0, 0, 0);                               \
  }
#define RSM_GEMM_STORE(BUF)                                                                \
  _Pragma("unroll") for (int j = 0; j < 4; ++j) {                                          \
    const int q = t + kThreads * j;                                                        \
    const int row = q >> 3, ch = q & 7;                                                    \
    *reinterpret_cast<uint4*>(&lds[BUF][0][row * kPitch + ch * 16]) = ra[j];               \
    *reinterpret_cast<uint4*>(&lds[BUF][1][row * kPitch + ch * 16]) = rb[j];               \
  }

  floatx16 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;

  const int n_k = (p.K + BK - 1) / BK;
  RSM_GEMM_LOAD(0);
  RSM_GEMM_STORE(0);
  __syncthreads();
  for (int kt = 0; kt < n_k; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < n_k) {
      RSM_GEMM_LOAD((kt + 1) * BK);
    }
    const unsigned char* la = lds[buf][0];
    const unsigned char* lb = lds[buf][1];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int off = (2 * g + lh) * 16;
      uint4 fa[2], fb[2];
#pragma unroll
      for (int i = 0; i < 2; ++i)
        fa[i] = *reinterpret_cast<const uint4*>(la + (wm + 32 * i + li) * kPitch + off);
#pragma unroll
      for (int j = 0; j < 2; ++j)
        fb[j] = *reinterpret_cast<const uint4*>(lb + (wn + 32 * j + li) * kPitch + off);
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = Mfma<T>::step(fa[i], fb[j], acc[i][j]);
    }
    if (kt + 1 < n_k) {
      RSM_GEMM_STORE(buf ^ 1);
    }
    __syncthreads();
  }
#undef RSM_GEMM_LOAD
#undef RSM_GEMM_STORE

  // 32x32 accumulator layout: element v of lane l is row 8(v/4) + 4(l/32) + v%4, column l%32
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wn + 32 * j + li;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = m0 + wm + 32 * i + 8 * (v >> 2) + 4 * lh + (v & 3);
        if (row < p.M && col < p.N) p.c[int64_t(row) * p.ldc + col] = acc[i][j][v];
      }
    }
}

// Large-tile variant: 256 x 256 outputs per workgroup of 4 waves, each wave
// owning a 128 x 128 block (4 x 4 MFMA tiles of 32 x 32, 256 accumulators).
// Pipeline (one workgroup per CU):
//  * LDS holds two k-tiles (2 x 73.7 KB): the matrix cores read one while the
//    other is refilled;
//  * one register staging set: during the first k-group of tile t it is
//    written to LDS (as tile t + 1) and at once reloaded with tile t + 2, so
//    each global load has a full tile of MFMAs to arrive;
//  * MFMA fragments are double-buffered: the LDS reads of the next k-group
//    are issued before the MFMAs of the current one;
//  * operands are read with raw buffer loads: a per-thread byte offset in
//    one VGPR plus a uniform offset (row block, k-tile) in an SGPR.  A read
//    past the operand's last byte returns zero, which pads the M / N tails;
//    k-chunks past K are sent out of range the same way.
// Every uniform offset (row block of rows up to m0 + 255, plus K) must stay
// below 2 GiB so that adding kOutOfRange cannot wrap (the launcher checks).
constexpr int kBig = 256;
constexpr uint32_t kBufferWord3 = 0x00020000;   // 32-bit data format, raw access
constexpr uint32_t kOutOfRange = 0x80000000u;

struct BigTile {
  __amdgpu_buffer_rsrc_t ra, rb;
  uint32_t va, vb;       // thread's byte offset within a 32-row block (B [K][N]: within an 8-row block)
  uint32_t sa, sb;       // bytes between consecutive 32-row blocks (B [K][N]: 8-row blocks)
  uint32_t a0, b0;       // byte offset of the tile's first row (B [K][N]: first column)
  uint32_t kbytes_thr;   // thread's k offset in bytes
  uint32_t kbytes;       // K in bytes
  uint32_t b_krow;       // B [K][N]: bytes between k rows
  uint32_t b_rr;         // B [K][N]: thread's row within an 8-row block
  uint32_t K;            // k extent in elements
};

// B stored [K][N] (BF16): a k-tile of B is 64 k rows x 256 columns, kept in
// LDS with that orientation at a row pitch of kPitchBN bytes (576 = 512 +
// 64: the four rows read by one 16-lane group of a transposing read start
// 64 bytes apart in the banks, and the two groups of a half-wave 32 bytes
// apart, so a half-wave touches every bank once).  MFMA B fragments (8
// consecutive k of one column per lane) come from two ds_read_b64_tr_b16:
// in each 16-lane group, lane L reads 4 columns at row kb + L / 4, column
// nb + 4 (L % 4), and lane i receives the 4 rows of column nb + i.
constexpr int kPitchBN = 576;
static_assert(64 * kPitchBN == kBig * kPitch, "B [K][N] tile must fill the B half of a k-tile buffer");

typedef short short4_t __attribute__((ext_vector_type(4)));

// Loads staging registers j in [J0, J0 + NJ) of both operands (rows
// (t >> 3) + 32 j of the tile) for the k-tile at byte offset k0_bytes.
template <int J0, int NJ, bool BN>
__device__ __forceinline__ void big_load(const BigTile& b, uint32_t k0_bytes, uint4 (&r)[16]) {
  const bool ok = k0_bytes + b.kbytes_thr < b.kbytes;
  const uint32_t va = ok ? b.va : kOutOfRange;
  const uint32_t vb = ok ? b.vb : kOutOfRange;
  const uint32_t k0 = k0_bytes / 2;   // B [K][N] is BF16
#pragma unroll
  for (int j = J0; j < J0 + NJ; ++j) {
    r[j] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(
                                         b.ra, va, b.a0 + j * b.sa + k0_bytes, 0));
    if (BN) {
      // k row k0 + rr + 8 j of columns n0 + 8 (t % 32) ..; rows past K read zero
      const uint32_t vbj = k0 + b.b_rr + 8u * uint32_t(j) < b.K ? b.vb : kOutOfRange;
      r[8 + j] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(
                                               b.rb, vbj, b.b0 + k0 * b.b_krow + j * b.sb, 0));
    } else {
      r[8 + j] = __builtin_bit_cast(uint4, __builtin_amdgcn_raw_buffer_load_b128(
                                               b.rb, vb, b.b0 + j * b.sb + k0_bytes, 0));
    }
  }
}

template <int J0, int NJ, bool BN>
__device__ __forceinline__ void big_store(unsigned char* buf, int t, const uint4 (&r)[16]) {
  constexpr int kOp = kBig * kPitch;
#pragma unroll
  for (int j = J0; j < J0 + NJ; ++j) {
    const int off = ((t >> 3) + 32 * j) * kPitch + (t & 7) * 16;
    *reinterpret_cast<uint4*>(buf + off) = r[j];
    const int off_b = BN ? ((t >> 5) + 8 * j) * kPitchBN + (t & 31) * 16 : off;
    *reinterpret_cast<uint4*>(buf + kOp + off_b) = r[8 + j];
  }
}

// Fragments of k-group g (16 k values): A rows (and B rows when B is stored
// Bt[n][k]) by 16-byte reads; B stored [K][N] by pairs of transposing reads
// from lane offset bfo (rows 8 lh + L / 4, columns wn + 16 ((lane / 16) % 2)
// + 4 (L % 4)).
template <bool BN>
__device__ __forceinline__ void big_frags(const unsigned char* la, int wm, int wn, int li, int lh, int bfo,
                                          int g, uint4 (&fa)[4], uint4 (&fb)[4]) {
  constexpr int kOp = kBig * kPitch;
  const int off = (2 * g + lh) * 16;
#pragma unroll
  for (int i = 0; i < 4; ++i) fa[i] = *reinterpret_cast<const uint4*>(la + (wm + 32 * i + li) * kPitch + off);
  if (BN) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const unsigned char* q = la + kOp + bfo + 16 * g * kPitchBN + 64 * j;
      const short4_t lo = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
          (__attribute__((address_space(3))) short4_t*)(q));
      const short4_t hi = __builtin_amdgcn_ds_read_tr16_b64_v4i16(
          (__attribute__((address_space(3))) short4_t*)(q + 4 * kPitchBN));
      const uint2 l2 = __builtin_bit_cast(uint2, lo), h2 = __builtin_bit_cast(uint2, hi);
      fb[j] = make_uint4(l2.x, l2.y, h2.x, h2.y);
    }
  } else {
#pragma unroll
    for (int j = 0; j < 4; ++j)
      fb[j] = *reinterpret_cast<const uint4*>(la + kOp + (wn + 32 * j + li) * kPitch + off);
  }
}

// MFMAs of one LDS k-tile.  With `refill` set, the staged tile is written
// there a quarter per k-group, each quarter right after that group's MFMAs
// are issued; each quarter of the staging set is then reloaded from k byte
// offset `k_next` (K bytes once no k-tile is left: all out of range).

// One k-group G of a k-tile: the 16 MFMAs of group G, with the LDS reads of
// group G + 1's fragments, a quarter of the refill (LDS writes of staged
// data) and the reload of that quarter slotted between them, one memory
// instruction after each MFMA.
template <typename T, int G, bool BN>
__device__ __forceinline__ void big_group(const unsigned char* la, unsigned char* refill, uint32_t k_next,
                                          const BigTile& bt, int t, uint4 (&stage)[16], int wm, int wn,
                                          int li, int lh, int bfo, uint4 (&fa)[2][4], uint4 (&fb)[2][4],
                                          floatx16 (&acc)[4][4]) {
  constexpr int c = G & 1;
  constexpr int kReads = BN ? 12 : 8;   // LDS read instructions per fragment set
  if (G < 3) big_frags<BN>(la, wm, wn, li, lh, bfo, G + 1, fa[c ^ 1], fb[c ^ 1]);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = Mfma<T>::step(fa[c][i], fb[c][j], acc[i][j]);
  big_store<2 * G, 2, BN>(refill, t, stage);
  big_load<2 * G, 2, BN>(bt, k_next, stage);
  // instruction classes: 0x008 MFMA, 0x020 VMEM read, 0x100 DS read, 0x200 DS write
  if (G < 3) {
#pragma unroll
    for (int k = 0; k < kReads; ++k) {
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    }
  }
  if (BN && G < 3) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    }
  } else {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      __builtin_amdgcn_sched_group_barrier(0x200, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      __builtin_amdgcn_sched_group_barrier(0x020, 1, 0);
      __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x008, G < 3 ? 0 : 8, 0);
  }
  __builtin_amdgcn_sched_barrier(0);
}

// MFMAs of one LDS k-tile.  The staged next tile is written to `refill` a
// quarter per k-group and each quarter of the staging set is reloaded from k
// byte offset `k_next` (K bytes once no k-tile is left: all out of range,
// and the writes then go to a buffer that is not read again).
template <typename T, bool BN>
__device__ __forceinline__ void big_compute(const unsigned char* la, unsigned char* refill, uint32_t k_next,
                                            const BigTile& bt, int t, uint4 (&stage)[16], int wm, int wn,
                                            int li, int lh, int bfo, floatx16 (&acc)[4][4]) {
  uint4 fa[2][4], fb[2][4];
  big_frags<BN>(la, wm, wn, li, lh, bfo, 0, fa[0], fb[0]);
  big_group<T, 0, BN>(la, refill, k_next, bt, t, stage, wm, wn, li, lh, bfo, fa, fb, acc);
  big_group<T, 1, BN>(la, refill, k_next, bt, t, stage, wm, wn, li, lh, bfo, fa, fb, acc);
  big_group<T, 2, BN>(la, refill, k_next, bt, t, stage, wm, wn, li, lh, bfo, fa, fb, acc);
  big_group<T, 3, BN>(la, refill, k_next, bt, t, stage, wm, wn, li, lh, bfo, fa, fb, acc);
}

// BN: B is stored [K][N] (p.ldb = elements between k rows, BF16 only).
template <typename T, bool BN>
__global__ void __launch_bounds__(kThreads, 1) gemm_tn_big_kernel(TnArgs p) {
  extern __shared__ __attribute__((aligned(16))) unsigned char dyn[];
  constexpr int kBuf = 2 * kBig * kPitch;   // one k-tile: A rows then B rows

  int tm, tn;
  tile_of(blockIdx.x, p.tiles_m, p.tiles_n, &tm, &tn);
  const int t = threadIdx.x;
  const int lane = t & 63, wave = t >> 6;
  const int wm = (wave >> 1) * 128, wn = (wave & 1) * 128;
  const int li = lane & 31, lh = lane >> 5;
  const int m0 = tm * kBig, n0 = tn * kBig;
  constexpr uint32_t S = sizeof(T);
  const uint32_t a_span = uint32_t((int64_t(p.M - 1) * p.lda + p.K) * S);
  const uint32_t b_span = BN ? uint32_t((int64_t(p.K - 1) * p.ldb + p.N) * S)
                             : uint32_t((int64_t(p.N - 1) * p.ldb + p.K) * S);
  BigTile bt;
  bt.ra = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p.a), short(0), int(a_span), int(kBufferWord3));
  bt.rb = __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p.b), short(0), int(b_span), int(kBufferWord3));
  bt.kbytes_thr = uint32_t(t & 7) * 16u;
  bt.va = uint32_t(t >> 3) * uint32_t(p.lda) * S + bt.kbytes_thr;
  bt.sa = 32u * uint32_t(p.lda) * S;
  bt.a0 = uint32_t(m0) * uint32_t(p.lda) * S;
  bt.kbytes = uint32_t(p.K) * S;
  bt.K = uint32_t(p.K);
  if (BN) {
    bt.b_rr = uint32_t(t >> 5);
    bt.b_krow = uint32_t(p.ldb) * S;
    bt.vb = bt.b_rr * bt.b_krow + uint32_t(t & 31) * 16u;
    bt.sb = 8u * bt.b_krow;
    bt.b0 = uint32_t(n0) * S;
  } else {
    bt.b_rr = 0;
    bt.b_krow = 0;
    bt.vb = uint32_t(t >> 3) * uint32_t(p.ldb) * S + bt.kbytes_thr;
    bt.sb = 32u * uint32_t(p.ldb) * S;
    bt.b0 = uint32_t(n0) * uint32_t(p.ldb) * S;
  }
  // transposing-read lane offset within the B half of a k-tile buffer
  const int L = lane & 15;
  const int bfo = (8 * lh + (L >> 2)) * kPitchBN + (wn + 16 * ((lane >> 4) & 1) + 4 * (L & 3)) * 2;

  floatx16 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 16; ++v) acc[i][j][v] = 0.0f;

  const int n_k = int((bt.kbytes + kRowBytes - 1) / kRowBytes);
  uint4 stage[16];
  big_load<0, 8, BN>(bt, 0, stage);
  big_store<0, 8, BN>(dyn, t, stage);
  if (n_k > 1) big_load<0, 8, BN>(bt, kRowBytes, stage);
  __syncthreads();
  for (int kt = 0; kt < n_k; ++kt) {
    const unsigned char* la = dyn + (kt & 1) * kBuf;
    unsigned char* refill = dyn + ((kt + 1) & 1) * kBuf;
    big_compute<T, BN>(la, refill, kt + 2 < n_k ? uint32_t(kt + 2) * kRowBytes : bt.kbytes, bt, t, stage, wm,
                       wn, li, lh, bfo, acc);
    __syncthreads();
  }

#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = n0 + wn + 32 * j + li;
#pragma unroll
      for (int v = 0; v < 16; ++v) {
        const int row = m0 + wm + 32 * i + 8 * (v >> 2) + 4 * lh + (v & 3);
        if (row < p.M && col < p.N) p.c[int64_t(row) * p.ldc + col] = acc[i][j][v];
      }
    }
}

// dst[c][r] = src[r][c] for a rows x cols matrix (element type E)
template <typename E>
__global__ void __launch_bounds__(256) transpose_kernel(const E* __restrict__ src, E* __restrict__ dst,
                                                        int rows, int cols, int64_t lds_src,
                                                        int64_t lds_dst) {
  __shared__ E tile[64][65];
  const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int r = ty; r < 64; r += 4) {
    const int gr = r0 + r, gc = c0 + tx;
    if (gr < rows && gc < cols) tile[r][tx] = src[int64_t(gr) * lds_src + gc];
  }
  __syncthreads();
  for (int c = ty; c < 64; c += 4) {
    const int gc = c0 + c, gr = r0 + tx;
    if (gr < rows && gc < cols) dst[int64_t(gc) * lds_dst + gr] = tile[tx][c];
  }
}

// The same with 16-byte accesses on both sides (V = 16 / sizeof(E) elements):
// a 64 x 64 tile is loaded row by row in 16-byte pieces into LDS (rows padded
// by one piece) and written column by column, each output piece gathering V
// elements of one LDS column.  Needs cols % V == 0, rows % V == 0 and
// 16-byte aligned bases (the launcher checks), so a piece is wholly in or
// out of range.
template <typename E>
__global__ void __launch_bounds__(256) transpose_vec_kernel(const E* __restrict__ src, E* __restrict__ dst,
                                                            int rows, int cols) {
  constexpr int V = 16 / int(sizeof(E));
  constexpr int P = 64 / V;         // pieces per tile row
  constexpr int R = 256 / P;        // tile rows per pass
  __shared__ __attribute__((aligned(16))) E tile[64][64 + V];
  const int r0 = blockIdx.y * 64, c0 = blockIdx.x * 64;
  const int piece = threadIdx.x % P, rr = threadIdx.x / P;
#pragma unroll
  for (int r = rr; r < 64; r += R) {
    const int gr = r0 + r, gc = c0 + piece * V;
    if (gr < rows && gc < cols)
      *reinterpret_cast<uint4*>(&tile[r][piece * V]) =
          *reinterpret_cast<const uint4*>(src + int64_t(gr) * cols + gc);
  }
  __syncthreads();
#pragma unroll
  for (int c = rr; c < 64; c += R) {
    const int gc = c0 + c, gr = r0 + piece * V;
    if (gc < cols && gr < rows) {
      E v[V];
#pragma unroll
      for (int i = 0; i < V; ++i) v[i] = tile[piece * V + i][c];
      *reinterpret_cast<uint4*>(dst + int64_t(gc) * rows + gr) = *reinterpret_cast<const uint4*>(v);
    }
  }
}

template <typename E>
hipError_t transpose(const void* src, void* dst, int rows, int cols, hipStream_t st) {
  constexpr int V = 16 / int(sizeof(E));
  dim3 grid((cols + 63) / 64, (rows + 63) / 64);
  if (cols % V == 0 && rows % V == 0 &&
      !((reinterpret_cast<uintptr_t>(src) | reinterpret_cast<uintptr_t>(dst)) & 15))
    transpose_vec_kernel<E><<<grid, 256, 0, st>>>(static_cast<const E*>(src), static_cast<E*>(dst), rows, cols);
  else
    transpose_kernel<E><<<grid, 256, 0, st>>>(static_cast<const E*>(src), static_cast<E*>(dst), rows, cols,
                                              cols, rows);
  return hipGetLastError();
}

}  // namespace

bool gemm_supported(const GemmArgs& a, int compute) {
  const int per = compute == RSM_BF16 ? 8 : 4;   // elements per 16-byte chunk
  if (a.M < 1 || a.N < 1 || a.K < 1) return false;
  if (a.K % per) return false;
  // the k-contiguous copies have row length K; both M and N strides must keep
  // 16-byte alignment of every row
  return true;
}

const char* gemm_variant_name(const GemmArgs& a, int compute) {
  const bool ta = a.a_sk != 1, tb = a.b_sk != 1;
  if (compute == RSM_BF16) {
    if (ta && tb) return "gemm_mfma_bf16_tt";
    if (ta) return "gemm_mfma_bf16_tn_at";
    if (tb) return "gemm_mfma_bf16_nn";
    return "gemm_mfma_bf16_nt";
  }
  if (ta && tb) return "gemm_mfma_f32_tt";
  if (ta) return "gemm_mfma_f32_tn_at";
  if (tb) return "gemm_mfma_f32_nn";
  return "gemm_mfma_f32_nt";
}

namespace {

// Kernel shape of a product: large tiles once the output has at least 200
// tiles of 256 x 256 and the large kernel's 32-bit buffer offsets reach;
// bn: BF16 B stored [K][N] with 16-byte aligned rows, read in place by the
// large kernel (transposing LDS reads) without a transposed copy (its
// offsets reach (K + 64) k rows plus N columns).
struct GemmShape {
  bool ta, tb, bn, big;
};

GemmShape gemm_shape(const GemmArgs& g, int compute, bool check_b_alignment) {
  GemmShape s{};
  const int64_t es = compute == RSM_BF16 ? 2 : 4;
  s.ta = g.a_sk != 1;
  s.tb = g.b_sk != 1;
  const bool big_shape = int64_t(g.M) * g.N >= int64_t(256) * 256 * 200;
  s.bn = compute == RSM_BF16 && s.tb && g.b_sn == 1 && big_shape &&
         !(check_b_alignment && (reinterpret_cast<uintptr_t>(g.b) & 15)) && !((g.b_sk * 2) & 15) &&
         (int64_t(g.K + 64) * g.b_sk + g.N) * 2 + 4096 < (int64_t(1) << 31);
  const int64_t lda = s.ta ? g.K : g.a_sm;
  const int64_t ldb = s.tb ? g.K : g.b_sn;
  const int64_t a_span = (int64_t(g.M + kBig) * lda + g.K) * es;
  const int64_t b_span = s.bn ? 0 : (int64_t(g.N + kBig) * ldb + g.K) * es;
  s.big = big_shape && a_span < (int64_t(1) << 31) && b_span < (int64_t(1) << 31);
  return s;
}

}  // namespace

int64_t gemm_lds_bytes_per_operand(const GemmArgs& g, int compute) {
  return gemm_shape(g, compute, false).big ? int64_t(2) * kBig * kPitch : int64_t(2) * kBM * kPitch;
}

int gemm_tile_side(const GemmArgs& g, int compute) { return gemm_shape(g, compute, false).big ? kBig : kBM; }

hipError_t launch_gemm(const GemmArgs& g, int compute, hipStream_t st) {
  (void)hipGetLastError();  // clear a stale error left by an unrelated earlier call
  const size_t es = compute == RSM_BF16 ? 2 : 4;
  const GemmShape shape = gemm_shape(g, compute, true);
  const bool ta = shape.ta, tb = shape.tb, bn = shape.bn;
  const size_t a_bytes = ta ? ((size_t(g.M) * g.K * es + 255) & ~size_t(255)) : 0;
  const size_t b_bytes = tb && !bn ? ((size_t(g.N) * g.K * es + 255) & ~size_t(255)) : 0;
  char* ws = nullptr;
  if (a_bytes + b_bytes) {
    rsm_status s;
    ws = static_cast<char*>(workspace(a_bytes + b_bytes, st, &s));
    if (s != RSM_OK) return hipErrorOutOfMemory;
  }
  TnArgs p;
  p.M = g.M;
  p.N = g.N;
  p.K = g.K;
  p.ldc = g.c_sm;
  p.c = g.c;
  p.a = g.a;
  p.lda = g.a_sm;
  p.b = g.b;
  p.ldb = g.b_sn;
  hipError_t e;
  if (ta) {  // A stored [K][M]: make A[m][k]
    e = es == 2 ? transpose<uint16_t>(g.a, ws, g.K, g.M, st) : transpose<float>(g.a, ws, g.K, g.M, st);
    if (e != hipSuccess) {
      fail(RSM_E_HIP, std::string("gemm: transpose of A failed: ") + hipGetErrorString(e));
      return e;
    }
    p.a = ws;
    p.lda = g.K;
  }
  if (bn) {
    p.ldb = g.b_sk;   // elements between k rows of B [K][N]
  } else if (tb) {  // B stored [K][N]: make Bt[n][k]
    e = es == 2 ? transpose<uint16_t>(g.b, ws + a_bytes, g.K, g.N, st)
                : transpose<float>(g.b, ws + a_bytes, g.K, g.N, st);
    if (e != hipSuccess) {
      fail(RSM_E_HIP, std::string("gemm: transpose of B failed: ") + hipGetErrorString(e));
      return e;
    }
    p.b = ws + a_bytes;
    p.ldb = g.K;
  }
  // 16-byte alignment of every row start of both operands
  if (((reinterpret_cast<uintptr_t>(p.a) | reinterpret_cast<uintptr_t>(p.b)) & 15) ||
      ((p.lda * es) & 15) || ((p.ldb * es) & 15)) {
    fail(RSM_E_HIP, "gemm: operand rows not 16-byte aligned (lda " + std::to_string(p.lda) +
                        ", ldb " + std::to_string(p.ldb) + ")");
    return hipErrorInvalidValue;
  }
  // large tiles: their buffer loads use 32-bit offsets, which must stay
  // below 2 GiB up to the last row of the last, padded 256-row block plus K
  const bool big = shape.big;
  if (bn && !big) {
    fail(RSM_E_HIP, "gemm: internal: [K][N] operand planned for the large-tile kernel");
    return hipErrorInvalidValue;
  }
  const int tile = big ? kBig : kBM;
  p.tiles_m = (g.M + tile - 1) / tile;
  p.tiles_n = (g.N + tile - 1) / tile;
  const int grid = p.tiles_m * p.tiles_n;
  const size_t lds_big = size_t(2) * 2 * kBig * kPitch;
  if (big) {
    if (compute == RSM_BF16 && bn) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm_tn_big_kernel<uint16_t, true>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_big));
      gemm_tn_big_kernel<uint16_t, true><<<grid, kThreads, lds_big, st>>>(p);
    } else if (compute == RSM_BF16) {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm_tn_big_kernel<uint16_t, false>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_big));
      gemm_tn_big_kernel<uint16_t, false><<<grid, kThreads, lds_big, st>>>(p);
    } else {
      (void)hipFuncSetAttribute(reinterpret_cast<const void*>(&gemm_tn_big_kernel<float, false>),
                                hipFuncAttributeMaxDynamicSharedMemorySize, int(lds_big));
      gemm_tn_big_kernel<float, false><<<grid, kThreads, lds_big, st>>>(p);
    }
  } else if (compute == RSM_BF16) {
    gemm_tn_kernel<uint16_t><<<grid, kThreads, 0, st>>>(p);
  } else {
    gemm_tn_kernel<float><<<grid, kThreads, 0, st>>>(p);
  }
  e = hipGetLastError();
  if (e != hipSuccess)
    fail(RSM_E_HIP, "gemm: kernel launch (grid " + std::to_string(grid) + ") failed: " +
                        hipGetErrorString(e));
  return e;
}

}  // namespace rsm
