// k_filter2d.hip -- k x k weighted windows with stride s on 2-D arrays.
//
// A workgroup of 256 threads (16 x 16) computes one tile of TH x TW outputs
// (TH = 16 RY, TW = 16 RX with RX S = 4).  The input region the tile's
// windows overlap, ((TH-1) S + K) x ((TW-1) S + K) elements, is staged in LDS
// once, with the modular wrap applied while loading (centred origins wrap on
// every border).  Each thread then computes an RY x RX block of outputs:
// every LDS row segment it needs (RX S + K - S floats, 16-byte aligned
// because RX S = 4) is read once with ds_read_b128 and used by each of its
// RX outputs and each of its RY output rows that the segment's row meets,
// so LDS traffic per output falls with RX and RY.  The k x k
// weights are uniform across the workgroup and read-only: they are read as
// constant memory through the scalar unit, one window row at a time, and
// the FMAs take them from scalar registers.
//
// Two launch forms share the tile body:
//  * filter2d_kernel: one problem, one workgroup per tile (plain launches);
//  * filter2d_persistent: a grid sized to the resident capacity walks a
//    host-built table of (problem, tile) entries round-robin: workgroup b
//    takes entries b, b + grid, ...  Each workgroup fetches the next entry
//    before running the current tile and loads that entry's problem
//    descriptor after it (a second descriptor held across the tile pushed
//    the kernel's scalar registers into memory spills and cost 15 %); there
//    is no atomic and nothing to reset between graph replays.
#include <hip/hip_runtime.h>

#include "rsm_internal.h"

namespace rsm {
namespace {

constexpr int kThreads = 256;
constexpr uint32_t kRawBuffer = 0x00020000;   // buffer resource word 3: 32-bit data, raw access
constexpr uint32_t kOutOfRange = 0x80000000u;  // a byte offset past every buffer here (< 2 GiB)

__host__ __device__ constexpr int rx_of(int S) { return 4 / S; }
__host__ __device__ constexpr int seg_of(int K, int S) { return (rx_of(S) - 1) * S + K; }
// floats read per row segment, rounded up to whole 16-byte vectors
__host__ __device__ constexpr int seg4_of(int K, int S) { return (seg_of(K, S) + 3) / 4; }
__host__ __device__ constexpr int lds_rows(int K, int S, int RY) { return (16 * RY - 1) * S + K; }
__host__ __device__ constexpr int lds_pitch(int K, int S) {
  // widest read: last thread's segment start (15 * RX * S = 60) + 4 * seg4
  return 60 + 4 * seg4_of(K, S) + 4;
}
__host__ __device__ constexpr int lds_cols(int K, int S) { return (16 * rx_of(S) - 1) * S + K; }
constexpr int kWPitch = 12;   // weights of one window row held per trip (K <= 9 of them)
__host__ __device__ constexpr int lds_floats(int K, int S, int RY) { return lds_rows(K, S, RY) * lds_pitch(K, S); }


__device__ __forceinline__ int mod_pos(int v, int n) {
  // v >= 0 here; reduce into [0, n)
  return v < n ? v : v % n;
}

// Frame and tile coordinates of tile `local` of problem p.
__device__ __forceinline__ void tile_pos(const Filter2DProblem& p, int64_t local, int* frame, int* ty, int* tx) {
  const uint32_t tiles_pf = uint32_t(p.tiles_per_frame);
  *frame = int(uint32_t(local) / tiles_pf);
  const int rem = int(uint32_t(local) - uint32_t(*frame) * tiles_pf);
  *ty = rem / p.tiles_w;
  *tx = rem - *ty * p.tiles_w;
}

template <int K, int S, int RY>
__device__ __forceinline__ void compute_tile(const Filter2DProblem& p, int64_t local, const float* lds) {
  constexpr int RX = rx_of(S);
  constexpr int TH = 16 * RY, TW = 16 * RX;
  constexpr int LR = lds_rows(K, S, RY), LP = lds_pitch(K, S);
  constexpr int SEG4 = seg4_of(K, S);
  int frame, ty, tx;
  tile_pos(p, local, &frame, &ty, &tx);
  // the k x k weights are the same for every thread of the tile and are not
  // written by the kernel: read as constant memory, they come through the
  // scalar unit into scalar registers, one window row at a time, and every
  // FMA takes its weight from there (no LDS reads for them)
  const __attribute__((address_space(4))) float* wc = (const __attribute__((address_space(4))) float*)(p.c);
  const int t = threadIdx.x;
  const int tr = t >> 4, tc = t & 15;
  float acc[RY][RX];
#pragma unroll
  for (int i = 0; i < RY; ++i)
#pragma unroll
    for (int j = 0; j < RX; ++j) acc[i][j] = 0.0f;
  // one LDS row per trip, read once: with stride S the thread's RY output
  // rows use the (RY - 1) S + K region rows from tr RY S on, and region row
  // r meets output row i through window row dy = r - i S when 0 <= dy < K
  // (a test uniform over the wave).  A row segment read once serves every
  // output row whose windows cover it (RY K segment reads become
  // (RY - 1) S + K), and each output still adds its window rows in
  // ascending order, so the sums do not change.  The loop is not unrolled:
  // one segment and the accumulators are live, not K x RY segments.
  constexpr int NRW = (RY - 1) * S + K;
  static_assert(15 * RY * S + NRW <= LR, "the last thread's rows lie inside the staged region");
  const float* base = lds + tr * RY * S * LP + tc * RX * S;
#pragma unroll 1
  for (int r = 0; r < NRW; ++r) {
    const float* row = base + r * LP;
    float seg[4 * SEG4];
#pragma unroll
    for (int v = 0; v < SEG4; ++v) {
      const float4 q = *reinterpret_cast<const float4*>(row + 4 * v);
      seg[4 * v + 0] = q.x; seg[4 * v + 1] = q.y; seg[4 * v + 2] = q.z; seg[4 * v + 3] = q.w;
    }
#pragma unroll
    for (int i = 0; i < RY; ++i) {
      const int dy = r - i * S;
      if (dy >= 0 && dy < K) {
        float w[kWPitch];
#pragma unroll
        for (int v = 0; v < K; ++v) w[v] = wc[dy * K + v];
#pragma unroll
        for (int j = 0; j < RX; ++j)
#pragma unroll
          for (int dx = 0; dx < K; ++dx) acc[i][j] = fmaf(w[dx], seg[j * S + dx], acc[i][j]);
      }
    }
  }
  // the frame's outputs as a raw buffer: an output past the array's edge
  // gets an offset past the buffer's end, and the hardware drops that store
  // (no branch per output)
  const __amdgpu_buffer_rsrc_t ry = __builtin_amdgcn_make_buffer_rsrc(
      p.y + int64_t(frame) * p.RH * p.RW, short(0), p.RH * p.RW * 4, int(kRawBuffer));
  const int oy0 = ty * TH + tr * RY, ox0 = tx * TW + tc * RX;
  // a thread's RX outputs of a row go out as one store when all lie inside
  // the row (buffer stores need 4-byte alignment only); a group cut by the
  // row's end stores its outputs one by one
  const bool full = ox0 + RX <= p.RW;
#pragma unroll
  for (int i = 0; i < RY; ++i) {
    const int oy = oy0 + i;
    if (RX == 4) {
      typedef __attribute__((ext_vector_type(4))) unsigned int u4;
      const u4 v = {__builtin_bit_cast(uint32_t, acc[i][0]), __builtin_bit_cast(uint32_t, acc[i][1]),
                    __builtin_bit_cast(uint32_t, acc[i][2]), __builtin_bit_cast(uint32_t, acc[i][3])};
      const uint32_t off = (oy < p.RH && full) ? uint32_t(oy * p.RW + ox0) * 4u : kOutOfRange;
      __builtin_amdgcn_raw_buffer_store_b128(v, ry, off, 0, 0);
    } else if (RX == 2) {
      typedef __attribute__((ext_vector_type(2))) unsigned int u2;
      const u2 v = {__builtin_bit_cast(uint32_t, acc[i][0]), __builtin_bit_cast(uint32_t, acc[i][RX - 1])};
      const uint32_t off = (oy < p.RH && full) ? uint32_t(oy * p.RW + ox0) * 4u : kOutOfRange;
      __builtin_amdgcn_raw_buffer_store_b64(v, ry, off, 0, 0);
    }
    if (RX == 1 || !full) {
#pragma unroll
      for (int j = 0; j < RX; ++j) {
        const int ox = ox0 + j;
        const uint32_t off = (oy < p.RH && ox < p.RW) ? uint32_t(oy * p.RW + ox) * 4u : kOutOfRange;
        __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, acc[i][j]), ry, off, 0, 0);
      }
    }
  }
}

// One tile with register staging (plain launches: one workgroup per tile).
template <int K, int S, int RY>
__device__ __forceinline__ void filter_tile(const Filter2DProblem p, int64_t local, float* lds) {
  constexpr int RX = rx_of(S);
  constexpr int TH = 16 * RY, TW = 16 * RX;
  constexpr int LR = lds_rows(K, S, RY), LC = lds_cols(K, S), LP = lds_pitch(K, S);

  int frame, ty, tx;
  tile_pos(p, local, &frame, &ty, &tx);

  // ---- stage the tile's input region, wrapping modulo the array shape ----
  // Wave rq stages rows rq, rq + 4, ... with lane l at columns l and l + 64.
  // Rows go out in chunks of CR, all loads of a chunk issued before any is
  // consumed.
  constexpr int NR = (LR + 3) / 4;          // rows per row group
  constexpr int NC = (LC + 63) / 64;        // column passes (1 or 2)
  constexpr int CR = NR < 8 ? NR : 8;       // rows per chunk
  constexpr int NCH = (NR + CR - 1) / CR;
  const int iy0 = p.oh + ty * TH * S;   // >= 0 (origin stored reduced)
  const int ix0 = p.ow + tx * TW * S;
  const int t = threadIdx.x;
  const int lane = t & 63;
  // the wave's row group: the same on every lane, so the row walk below
  // (row indices, wrapping, row base addresses, the row bound) runs on the
  // scalar unit and each load takes a scalar base plus a 32-bit lane offset
  const int rq = __builtin_amdgcn_readfirstlane(t >> 6);
  const bool interior = iy0 + LR <= p.H && ix0 + LC <= p.W;
  float* ldst = lds + rq * LP + lane;
  // lanes past the region's last column load its last element instead (same
  // cache lines) and store nothing
  const bool col0 = LC >= 64 || lane < LC;
  const bool col1 = NC > 1 && lane + 64 < LC;
  const int l0 = col0 ? lane : LC - 1;
  const int l1 = col1 ? lane + 64 : LC - 1;
  // the staging loads are the tile's latency chain: while a wave issues
  // them it outranks the waves of other workgroups on the CU that are
  // computing (the batch runs about 7 % faster)
  __builtin_amdgcn_s_setprio(2);
  // The frame is read as a raw buffer (frames under 2 GiB, a planner
  // condition): a load takes the row's byte offset in a scalar register and
  // the lane's in a 32-bit vector register, with no 64-bit address arithmetic.
  const __amdgpu_buffer_rsrc_t rx = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(p.x + int64_t(frame) * p.H * p.W), short(0), p.H * p.W * 4, int(kRawBuffer));
  uint32_t c0, c1;
  int rowi;   // array row of the wave's next region row (border tiles)
  if (interior) {
    c0 = uint32_t(ix0 + l0) * 4u;
    c1 = uint32_t(ix0 + l1) * 4u;
    rowi = iy0 + rq;
  } else {
    c0 = uint32_t(mod_pos(ix0 + l0, p.W)) * 4u;
    c1 = uint32_t(mod_pos(ix0 + l1, p.W)) * 4u;
    rowi = mod_pos(iy0 + rq, p.H);
  }
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    float v[CR][NC];
#pragma unroll
    for (int i = 0; i < CR; ++i) {
      const int r = rq + 4 * (ch * CR + i);
      if (r < LR) {
        const int rowb = rowi * p.W * 4;
        v[i][0] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rx, c0, rowb, 0));
        if (NC > 1) v[i][NC - 1] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rx, c1, rowb, 0));
        // next row of this wave: 4 further, wrapped (border tiles only)
        rowi += 4;
        if (!interior)
          while (rowi >= p.H) rowi -= p.H;
      }
    }
    if (ch == 0) __syncthreads();  // the previous tile's readers are done with LDS
#pragma unroll
    for (int i = 0; i < CR; ++i) {
      const int r = rq + 4 * (ch * CR + i);
      if (r < LR) {
        if (col0) ldst[4 * (ch * CR + i) * LP] = v[i][0];
        if (NC > 1 && col1) ldst[4 * (ch * CR + i) * LP + 64] = v[i][NC - 1];
      }
    }
  }
  __builtin_amdgcn_s_setprio(0);
  __syncthreads();

  compute_tile<K, S, RY>(p, local, lds);
}

// RY for tile class tc of stride S.  LDS per workgroup stays under 22 KB so
// that seven workgroups fit in a CU's 160 KB.
__host__ __device__ constexpr int ry_of(int S, int tc) {
  return S == 4 ? 1 : S == 2 ? (tc == 0 ? 1 : 2) : (tc == 0 ? 1 : tc == 1 ? 2 : 4);
}

template <int K, int S, int RY>
__global__ void __launch_bounds__(kThreads) filter2d_kernel(Filter2DProblem p) {
  extern __shared__ float lds[];
  filter_tile<K, S, RY>(p, blockIdx.x, lds);
}

template <int K>
__device__ __forceinline__ void tile_s(const Filter2DProblem& p, int64_t local, float* lds) {
  switch (p.s) {
    case 1:
      if (ry_of(1, p.tc) == 1) filter_tile<K, 1, 1>(p, local, lds);
      else if (ry_of(1, p.tc) == 2) filter_tile<K, 1, 2>(p, local, lds);
      else filter_tile<K, 1, 4>(p, local, lds);
      break;
    case 2:
      if (ry_of(2, p.tc) == 1) filter_tile<K, 2, 1>(p, local, lds);
      else filter_tile<K, 2, 2>(p, local, lds);
      break;
    default: filter_tile<K, 4, 1>(p, local, lds); break;
  }
}

__device__ __forceinline__ void tile_any(const Filter2DProblem& p, int64_t local, float* lds) {
  switch (p.k) {
    case 3: tile_s<3>(p, local, lds); break;
    case 5: tile_s<5>(p, local, lds); break;
    case 7: tile_s<7>(p, local, lds); break;
    default: tile_s<9>(p, local, lds); break;
  }
}

// Persistent form: workgroup b takes table entries b, b + grid, ...; the
// next entry is fetched before the current tile runs, its descriptor after.  Each tile issues its staging loads before the barrier that waits
// for the previous tile's LDS readers.  The grid must not exceed the
// resident capacity (the launcher sizes it from the occupancy), so no
// workgroup starts late.
__global__ void __launch_bounds__(kThreads, 7) filter2d_persistent(const Filter2DProblem* __restrict__ probs,
                                                                   const uint2* __restrict__ tiles,
                                                                   int64_t n_tiles) {
  extern __shared__ float lds[];
  int64_t t = blockIdx.x;
  if (t >= n_tiles) return;
  uint2 e = tiles[t];
  Filter2DProblem p = probs[e.x];
  while (true) {
    const int64_t tn = t + gridDim.x;
    const bool more = tn < n_tiles;
    uint2 en = e;
    if (more) en = tiles[tn];
    tile_any(p, e.y, lds);
    if (!more) break;
    t = tn;
    e = en;
    p = probs[e.x];
  }
}

template <int K, int S>
hipError_t launch_ks(const Filter2DProblem& p, int64_t n_tiles, hipStream_t st) {
  switch (p.tc) {
    case 0: {
      constexpr int RY = ry_of(S, 0);
      filter2d_kernel<K, S, RY><<<unsigned(n_tiles), kThreads, lds_floats(K, S, RY) * 4, st>>>(p);
      break;
    }
    case 1: {
      constexpr int RY = ry_of(S, 1);
      filter2d_kernel<K, S, RY><<<unsigned(n_tiles), kThreads, lds_floats(K, S, RY) * 4, st>>>(p);
      break;
    }
    default: {
      constexpr int RY = ry_of(S, 2);
      filter2d_kernel<K, S, RY><<<unsigned(n_tiles), kThreads, lds_floats(K, S, RY) * 4, st>>>(p);
      break;
    }
  }
  return hipGetLastError();
}

template <int K>
hipError_t launch_k(const Filter2DProblem& p, int64_t n_tiles, hipStream_t st) {
  switch (p.s) {
    case 1: return launch_ks<K, 1>(p, n_tiles, st);
    case 2: return launch_ks<K, 2>(p, n_tiles, st);
    default: return launch_ks<K, 4>(p, n_tiles, st);
  }
}

}  // namespace

bool filter2d_supported(int k, int s) {
  return (k == 3 || k == 5 || k == 7 || k == 9) && (s == 1 || s == 2 || s == 4);
}

int filter2d_tile_rows(int s, int tc) { return 16 * ry_of(s, tc); }
int filter2d_tile_cols(int s) { return 16 * rx_of(s); }

size_t filter2d_lds_bytes(int k, int s, int tc) {
  return size_t(lds_floats(k, s, ry_of(s, tc))) * 4;
}

int filter2d_buf_floats(int k, int s, int tc) { return lds_floats(k, s, ry_of(s, tc)); }

// Fills the tiling fields of p for tile class tc (0..2).
void filter2d_set_tiles(Filter2DProblem* p, int tc) {
  p->tc = tc;
  p->tile_h = filter2d_tile_rows(p->s, tc);
  p->tile_w = filter2d_tile_cols(p->s);
  p->tiles_w = (p->RW + p->tile_w - 1) / p->tile_w;
  const int tiles_h = (p->RH + p->tile_h - 1) / p->tile_h;
  p->tiles_per_frame = tiles_h * p->tiles_w;
  p->n_tiles = int64_t(p->tiles_per_frame) * p->frames;
}

hipError_t launch_filter2d(const Filter2DProblem& p, hipStream_t st) {
  if (p.n_tiles <= 0) return hipSuccess;
  switch (p.k) {
    case 3: return launch_k<3>(p, p.n_tiles, st);
    case 5: return launch_k<5>(p, p.n_tiles, st);
    case 7: return launch_k<7>(p, p.n_tiles, st);
    default: return launch_k<9>(p, p.n_tiles, st);
  }
}

// Resident workgroups of the persistent kernel with an LDS buffer of
// buf_floats, times the CU count.
int filter2d_persistent_grid(int buf_floats) {
  int dev = 0, cus = 256, per_cu = 0;
  if (hipGetDevice(&dev) == hipSuccess) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      cus = v;
  }
  const size_t lds = size_t(buf_floats) * sizeof(float);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, reinterpret_cast<const void*>(&filter2d_persistent),
                                                   kThreads, lds) != hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return per_cu * cus;
}

hipError_t launch_filter2d_persistent(const Filter2DProblem* d_probs, const void* d_tiles, int64_t n_tiles,
                                      int grid, int buf_floats, hipStream_t st) {
  const size_t lds = size_t(buf_floats) * sizeof(float);
  filter2d_persistent<<<grid, kThreads, lds, st>>>(d_probs, static_cast<const uint2*>(d_tiles), n_tiles);
  return hipGetLastError();
}

}  // namespace rsm
