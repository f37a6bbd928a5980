// rollout.hpp -- device side of Alg. 1 for one tile of particles of one human:
// (beta, g) draw from the belief, H Boltzmann-heading lattice steps held in
// registers, and per-step emplacement through an LDS-privatised histogram
// window flushed to the global uint32 grid with coalesced atomics.
#pragma once

#include "common.hpp"

namespace capred {

// Everything the rollout needs about one human (trivially copyable; passed by
// value to the single-human kernel and stored in device memory for batches).
struct RolloutDesc {
  int32_t N, H, K, B, G, nx, ny;
  int32_t S;                // speeds (controls u = s K + k, U = S K)
  int32_t s_last;           // last allowed speed
  uint32_t smask;           // allowed speeds of the prediction (bit s)
  int32_t X0, Y0;           // start on the lattice (grid frame)
  int32_t Rx, Ry;           // max |S_kx|, |S_ky|: reach per step, lattice units
  uint32_t human, cycle;
  int32_t shift;            // 1: subtract the largest exponent (large beta * step)
  int32_t sym;              // 1: S_{k+K/2} = -S_k for every k < K/2 (K even)
  HeadingTable T;           // lattice-unit steps (exact integers) and squared lengths (FP32)
  float ibeta[CAP_MAX_B];   // 1 / (-beta q log2(e)), q = lattice pitch
  int32_t GX[CAP_MAX_G], GY[CAP_MAX_G];
  const double* belief;     // [G][B]
  uint32_t* counts;         // [H][ny][nx]
  uint32_t* offgrid;        // [H] or null
  uint8_t* trace_k;         // [N][H] or null
  int32_t* trace_pair;      // [N] or null
};

struct TileShared {
  double P[CAP_MAX_J];      // pair CDF (sequential FP64 prefix sums)
  int2 S[CAP_MAX_K];        // lattice steps for the dynamic heading index (one speed)
  int2 goal[CAP_MAX_G];
  float ibeta[CAP_MAX_B];
  uint32_t off[2];          // off-grid counters of the two in-flight steps
  uint32_t ntouch[3];       // first-touched window words per step (rotating)
  int last_pos;
};

__device__ __forceinline__ int64_t floor_shift16(int64_t v) { return v >> kLatticeShift; }

// Histogram window of step t: every particle is within t * (Rx, Ry) lattice
// units of the start, so its cell lies in [floor((X0 - tRx)/2^16),
// floor((X0 + tRx)/2^16)] (clipped to the grid).  Uniform across the block.
struct Window {
  int x0, y0, w, h;
};

// Reach window of step t for a start (X0, Y0) on the lattice.
__device__ __forceinline__ Window step_window_at(const RolloutDesc& d, int32_t X0, int32_t Y0,
                                                 int t) {
  // 64-bit only for the reach t * R (up to 2^36); the shifted bounds fit 32 bits,
  // so the clamps stay in scalar 32-bit arithmetic
  const int64_t rx = (int64_t)t * d.Rx, ry = (int64_t)t * d.Ry;
  int lx = (int)floor_shift16((int64_t)X0 - rx), hx = (int)floor_shift16((int64_t)X0 + rx);
  int ly = (int)floor_shift16((int64_t)Y0 - ry), hy = (int)floor_shift16((int64_t)Y0 + ry);
  lx = max(lx, 0);
  ly = max(ly, 0);
  hx = min(hx, d.nx - 1);
  hy = min(hy, d.ny - 1);
  Window win;
  win.x0 = lx;
  win.y0 = ly;
  win.w = hx >= lx ? hx - lx + 1 : 0;
  win.h = hy >= ly ? hy - ly + 1 : 0;
  return win;
}

__device__ __forceinline__ Window step_window(const RolloutDesc& d, int t) {
  return step_window_at(d, d.X0, d.Y0, t);
}

__device__ __forceinline__ uint32_t pick_word(const uint4& w, int s) {
  return s == 0 ? w.x : (s == 1 ? w.y : (s == 2 ? w.z : w.w));
}

// LDS bytes of the histogram window of one block: two window buffers of
// `cap` words (two 16-bit cell counters per word) and two lists of the words
// first touched in a step (16-bit word indices, one per particle at most).
// A step whose window needs more than `cap` words (and at most 2 cap) uses
// both buffers as one and the first list.
__host__ __device__ constexpr size_t window_lds_bytes(int cap, int particles_per_tile) {
  return (size_t)2 * cap * sizeof(uint32_t) + (size_t)2 * particles_per_tile * sizeof(uint16_t);
}

// Processes particles [first, first + P * blockDim.x) of human d (clipped to N).
// win: window_lds_bytes(cap, P * blockDim.x) bytes of LDS, zero on entry and
// on exit (cap <= 65536).  A step's window is flushed from the list of words
// its particles touched first, so the flush costs one entry per occupied
// word, whatever the window's area.  Windows of up to cap words alternate
// between the two buffers, so that a step's binning overlaps the previous
// step's flush; windows of up to 2 cap words (and 2^16 words, the reach of a
// list entry) take both buffers and wait at one more barrier for the previous
// flush; larger windows bin with global atomics.
//
// MS (several speeds): draw_control over the S K controls; `ctl` is an LDS
// array of CAP_MAX_U float4 that receives (fx, fy, s2) of every control, read
// per lane for the block recomputation and the step (unused otherwise).
//
// PAIR: draw the particles two at a time (draw_headings with M = 2), for fixed K of
// at most 16 without the shifted exponent, where the two chains fit in the
// registers of four waves per SIMD without spilling.
template <int KT, int P, bool SHIFT, bool MS, bool PAIR>
__device__ __forceinline__ void rollout_tile_body(const RolloutDesc& d, int64_t first,
                                                  uint32_t seed_lo, uint32_t seed_hi,
                                                  TileShared& sh, uint32_t* win, int cap,
                                                  float4* ctl) {
  const int tid = threadIdx.x;
  const int nthr = blockDim.x;
  const int J = d.G * d.B;
  // ---- shared tables
  if (tid == 0) {
    double acc = 0.0;
    int last = 0;
    for (int j = 0; j < J; ++j) {
      const double b = as_global(d.belief)[j];
      acc += b;
      sh.P[j] = acc;
      if (b > 0.0) last = j;
    }
    sh.last_pos = last;
    sh.off[0] = 0u;
    sh.off[1] = 0u;
    sh.ntouch[0] = sh.ntouch[1] = sh.ntouch[2] = 0u;
  }
  if constexpr (MS) {
    for (int u = tid; u < d.K * d.S; u += nthr)
      ctl[u] = make_float4(d.T.fx[u], d.T.fy[u], d.T.s2[u], 0.f);
  } else {
    for (int k = tid; k < d.K; k += nthr) sh.S[k] = make_int2((int)d.T.fx[k], (int)d.T.fy[k]);
  }
  for (int g = tid; g < d.G; g += nthr) sh.goal[g] = make_int2(d.GX[g], d.GY[g]);
  for (int b = tid; b < d.B; b += nthr) sh.ibeta[b] = d.ibeta[b];
  __syncthreads();

  // ---- per-particle (beta, g) draw, held for the whole horizon
  const uint32_t c3_pair = 2u * d.cycle, c3_head = 2u * d.cycle + 1u;
  int64_t idx[P];
  bool act[P];
  int32_t X[P], Y[P], GXp[P], GYp[P];
  float ib[P];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    idx[p] = first + (int64_t)p * nthr + tid;
    act[p] = idx[p] < d.N;
    X[p] = d.X0;
    Y[p] = d.Y0;
    GXp[p] = 0;
    GYp[p] = 0;
    ib[p] = 1.f;
    if (act[p]) {
      const uint4 w = philox10((uint32_t)idx[p], 0u, d.human, c3_pair, seed_lo, seed_hi);
      const double u = uniform24d(w.x);
      int lo = 0, hi = J;
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (sh.P[mid] > u) hi = mid;
        else lo = mid + 1;
      }
      const int j = lo < J ? lo : sh.last_pos;
      const int g = j / d.B, b = j - g * d.B;
      GXp[p] = sh.goal[g].x;
      GYp[p] = sh.goal[g].y;
      ib[p] = sh.ibeta[b];
      if (d.trace_pair) as_global(d.trace_pair)[idx[p]] = j;
    }
  }

  const size_t plane = (size_t)d.nx * (size_t)d.ny;
  uint4 rw[P];
  const int list_cap = P * nthr;
  uint16_t* lists = reinterpret_cast<uint16_t*>(win + 2 * cap);
  int m3 = 1;  // t mod 3
  for (int t = 1; t <= d.H; ++t, m3 = (m3 == 2 ? 0 : m3 + 1)) {
    const int s = (t - 1) & 3;
    if (s == 0) {
      // The round keys (key + r * Weyl constant) are derived from the seed here,
      // by scalar adds in every block, rather than held across the loop: kept,
      // they would pin 20 scalar registers that the step's other uniform values
      // need (the overflow goes to vector-register lanes, one VALU access each).
      uint32_t klo = seed_lo, khi = seed_hi;
      asm volatile("" : "+s"(klo), "+s"(khi));
#pragma unroll
      for (int p = 0; p < P; ++p)
        rw[p] = philox10((uint32_t)idx[p], (uint32_t)((t - 1) >> 2), d.human, c3_head, klo, khi);
    }
    const Window wd = step_window(d, t);
    // two 16-bit counters per LDS word (a tile never holds 65536 particles);
    // rows padded to an even number of cells
    const int half_w = (wd.w + 1) >> 1;
    const int words = half_w * wd.h;
    const bool single = words > cap && words <= 2 * cap && words <= 65536;
    const bool lds_mode = words <= cap || single;
    uint32_t* buf = single ? win : win + (t & 1) * cap;
    uint16_t* list = single ? lists : lists + (t & 1) * list_cap;
    // both buffers: the previous step's flush (of either buffer) must be over
    if (single) __syncthreads();
    uint32_t* grid_t = d.counts + (size_t)(t - 1) * plane;
    bool off_any = false;
    // Draws of all P particles first, then their emplacement: the draws are
    // independent dependency chains (transcendental latency), which the
    // scheduler can interleave only while no branch separates them.  Each
    // particle's step word is rw[p].x; the remaining words move down, so the
    // word is picked without branching on the step's phase.
    int kk[P];
    if constexpr (PAIR) {
      static_assert(P % 2 == 0 && !MS, "paired draws need an even P and one speed");
#pragma unroll
      for (int p = 0; p < P; p += 2) {
        float ax[2], ay[2], ibm[2], um[2];
        int ko[2];
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          ax[m] = (float)(X[p + m] - GXp[p + m]);
          ay[m] = (float)(Y[p + m] - GYp[p + m]);
          ibm[m] = ib[p + m];
          um[m] = uniform24f(rw[p + m].x);
          rw[p + m] = make_uint4(rw[p + m].y, rw[p + m].z, rw[p + m].w, 0u);
        }
        draw_headings<KT, SHIFT, 2>(ax, ay, ibm, um, d.T, ko);
#pragma unroll
        for (int m = 0; m < 2; ++m) {
          const int2 st = sh.S[ko[m]];
          X[p + m] += st.x;
          Y[p + m] += st.y;
          kk[p + m] = ko[m];
        }
      }
    } else {
#pragma unroll
      for (int p = 0; p < P; ++p) {
        // computed for inactive lanes too (harmless state), so that the P
        // particles stay in one basic block; only emplacement is predicated
        const float u = uniform24f(rw[p].x);
        rw[p] = make_uint4(rw[p].y, rw[p].z, rw[p].w, 0u);
        int k;
        if constexpr (MS)
          k = draw_control<KT, SHIFT>((float)(X[p] - GXp[p]), (float)(Y[p] - GYp[p]), ib[p], u,
                                      d.T, d.S, d.smask, d.s_last, ctl);
        else
          k = draw_heading<KT, SHIFT>((float)(X[p] - GXp[p]), (float)(Y[p] - GYp[p]), ib[p], u,
                                      d.T, d.K);
        if constexpr (MS) {
          const float4 c = ctl[k];
          X[p] += (int32_t)c.x;
          Y[p] += (int32_t)c.y;
        } else {
          const int2 st = sh.S[k];
          X[p] += st.x;
          Y[p] += st.y;
        }
        kk[p] = k;
      }
    }
    // The draws' results are fixed here (an empty asm that reads and writes
    // them), so that the compiler does not sink each draw into the branchy
    // emplacement of its particle below.
#pragma unroll
    for (int p = 0; p < P; ++p) asm volatile("" : "+v"(X[p]), "+v"(Y[p]), "+v"(kk[p]));
#pragma unroll
    for (int p = 0; p < P; ++p) {
      bool off = false;
      const int k = kk[p];
      bool fresh = false;     // this lane turned an empty window word non-empty
      uint32_t widx = 0;
      if (act[p]) {
        if (d.trace_k) as_global(d.trace_k)[(size_t)idx[p] * d.H + (t - 1)] = (uint8_t)k;
        const int cx = X[p] >> kLatticeShift, cy = Y[p] >> kLatticeShift;
        if (lds_mode) {
          // the particle's cell lies in the unclipped reach window, so it is on
          // the grid exactly when it lies in the clipped window
          const unsigned lx = (unsigned)(cx - wd.x0), ly = (unsigned)(cy - wd.y0);
          if (lx < (unsigned)wd.w && ly < (unsigned)wd.h) {
            widx = __umul24(ly, (unsigned)half_w) + (lx >> 1);  // both below 2^24
            fresh = atomicAdd(buf + widx, 1u << ((lx & 1u) << 4)) == 0u;
          } else {
            off = true;
          }
        } else if ((unsigned)cx < (unsigned)d.nx && (unsigned)cy < (unsigned)d.ny) {
          global_add(grid_t + (size_t)cy * d.nx + cx, 1u);
        } else {
          off = true;
        }
      }
      // append of the freshly touched words and the off-grid count: the
      // compiler's atomic optimizer turns each uniform-address increment into
      // one LDS atomic per wavefront plus a lane prefix count
      if (fresh) list[atomicAdd(&sh.ntouch[m3], 1u)] = (uint16_t)widx;
      off_any |= off;
      if (off) atomicAdd(&sh.off[t & 1], 1u);
    }
    (void)off_any;
    __syncthreads();
    // ---- flush the touched words of step t's window, clear them
    if (lds_mode) {
      // Word w of the window is row ry = floor(w / half_w), cells 2 rx and 2 rx + 1
      // with rx = w - ry half_w.  ry = trunc((w + 1/2) * fl(1/half_w)) exactly:
      // (w + 1/2) / half_w lies at least 1/(2 half_w) from an integer, while the
      // two roundings (reciprocal within 1 ulp, product) move it by at most
      // 2^-22 (w + 1/2) / half_w <= 2^-22 * 65536 / half_w, since w < 2^16.
      const float rhw = fast_rcp((float)half_w), hrhw = 0.5f * rhw;
      // byte offset of the window's first cell within the step's plane (< 2^30)
      const uint32_t base4 = 4u * ((uint32_t)wd.y0 * (uint32_t)d.nx + (uint32_t)wd.x0);
      const uint32_t nx4 = 4u * (uint32_t)d.nx;
      char* gbase = reinterpret_cast<char*>(grid_t);
      const uint32_t nt = sh.ntouch[m3];
      for (uint32_t i = tid; i < nt; i += nthr) {
        const uint32_t w = list[i];
        const uint32_t v = buf[w];
        buf[w] = 0u;
        const uint32_t ry = (uint32_t)fmaf((float)w, rhw, hrhw);
        const uint32_t rx = w - __umul24(ry, (uint32_t)half_w);
        const uint32_t off4 = __umul24(ry, nx4) + base4 + (rx << 3);
        uint32_t* g = reinterpret_cast<uint32_t*>(gbase + off4);
        const uint32_t lo = v & 0xFFFFu, hi = v >> 16;
        if (lo) global_add(g, lo);
        if (hi) global_add(g + 1, hi);
      }
    }
    if (tid == 0) {
      const uint32_t v = sh.off[t & 1];
      if (v && d.offgrid) global_add(d.offgrid + (t - 1), v);
      sh.off[t & 1] = 0u;
      // the list counter of step t-1 was read before this step's barrier and
      // is next appended to at step t+2, after the next barrier
      sh.ntouch[m3 == 0 ? 2 : m3 - 1] = 0u;
    }
  }
  __syncthreads();
}

// A tile of one human.  The shifted exponent is a property of the human
// (d.shift: beta * step too large for the unshifted exp2), not of the launch:
// a launch compiled with SHIFT also carries the unshifted body and takes it,
// uniformly per tile, for humans that do not need the shift, so that their
// draws are the same bits whichever humans share the launch.
template <int KT, int P, bool SHIFT, bool MS>
__device__ __forceinline__ void rollout_tile(const RolloutDesc& d, int64_t first, uint32_t seed_lo,
                                             uint32_t seed_hi, TileShared& sh, uint32_t* win,
                                             int cap, float4* ctl) {
  if constexpr (SHIFT) {
    if (!d.shift) {
      rollout_tile_body<KT, P, false, MS, false>(d, first, seed_lo, seed_hi, sh, win, cap, ctl);
      return;
    }
  }
  constexpr bool kPair = !SHIFT && !MS && KT > 0 && KT <= 16 && P % 2 == 0;
  rollout_tile_body<KT, P, SHIFT, MS, kPair>(d, first, seed_lo, seed_hi, sh, win, cap, ctl);
}

}  // namespace capred
