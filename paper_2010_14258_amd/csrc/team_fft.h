// Register-resident FFT of one power-of-two length L = 2^LOG2L (16 <= L <= 4096) carried out by a
// "team" of T = L/16 lanes of a workgroup, 16 complex values per lane.
//
// Element e of the sequence lives in lane (e mod T) of the team, register e / T; this layout is the
// same on input and on output, so global loads and stores of consecutive lanes touch consecutive
// elements.  The transform is a sequence of self-sorting Stockham stages of radix min(16, remaining):
// a stage with Ns = product of the earlier radices takes butterfly b = t + T i (i < 16/RAD) from
// registers i + r 16/RAD, multiplies by W_{Ns RAD}^{r (b mod Ns)}, runs the RAD-point DFT in
// registers and sends output r to position (b - b mod Ns) RAD + b mod Ns + r Ns.  Every stage but the
// last exchanges through LDS (write, barrier, read back in the lane layout, barrier); in the last stage
// the output positions coincide with the lane layout, so it stays in registers.  L = 256 therefore
// costs one LDS exchange, L = 4096 two.
//
// Twiddles W_L^k come from a table in LDS, built in FP64 and rounded once: the full table for L <= 256,
// otherwise two levels (W_L^k for k < 2^LB, then W_L^(k 2^LB)) whose product is taken in R.
#pragma once

#include "common.h"
#include "fft.h"

namespace ldbp {

constexpr int kTeamLanes = 16;  // values per lane

__host__ __device__ constexpr int team_tw_lb(int log2l) { return log2l <= 8 ? log2l : (log2l + 1) / 2; }
__host__ __device__ constexpr int team_tw_entries(int log2l) {
  return log2l <= 8 ? (1 << log2l) : (1 << team_tw_lb(log2l)) + (1 << (log2l - team_tw_lb(log2l)));
}

template <typename R, int LOG2L>
__device__ __forceinline__ cx_t<R> team_tw(int e, const cx_t<R>* tw) {
  if constexpr (LOG2L <= 8) {
    return tw[e];
  } else {
    constexpr int LB = team_tw_lb(LOG2L);
    const cx_t<R> a = tw[e & ((1 << LB) - 1)];
    const cx_t<R> b = tw[(1 << LB) + (e >> LB)];
    return cx_t<R>{a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
  }
}

// LDS exchange layouts.  Both are addressed by (position in the sequence, team index in the workgroup).
// Interleaved: position-major, teams fastest (used when consecutive lanes belong to different teams);
// a pad of `pad` elements every 16 positions spreads the stage writes over the banks.
template <typename V>
struct XchInterleaved {
  V* base;
  int teams, pad, g;
  __device__ __forceinline__ int at(int pos) const { return pos * teams + g + (pos >> 4) * pad; }
  __device__ __forceinline__ void put(int pos, V v) const { base[at(pos)] = v; }
  __device__ __forceinline__ V get(int pos) const { return base[at(pos)]; }
};

// Team-major: each team owns a row of `stride` elements (L + 16); positions are XOR-swizzled in their
// low five bits by bits 4..8 so that stage writes (stride 16 apart) and lane-layout reads both spread
// over the banks.  Needs L >= 32.
template <typename V>
struct XchTeamMajor {
  V* base;
  int stride, g;
  __device__ __forceinline__ int at(int pos) const { return g * stride + (pos ^ ((pos >> 4) & 31)); }
  __device__ __forceinline__ void put(int pos, V v) const { base[at(pos)] = v; }
  __device__ __forceinline__ V get(int pos) const { return base[at(pos)]; }
};

template <typename R, int DIR, int LOG2L, int NS_LOG, class Xch>
__device__ __forceinline__ void team_fft_from(cx_t<R> (&v)[kTeamLanes], int t, const Xch& xc,
                                              const cx_t<R>* tw) {
  using V = cx_t<R>;
  constexpr int REM = LOG2L - NS_LOG;
  constexpr int RAD_LOG = REM < 4 ? REM : 4;
  constexpr int RAD = 1 << RAD_LOG;
  constexpr int NB = kTeamLanes / RAD;
  constexpr int NS = 1 << NS_LOG;
  constexpr int T = 1 << (LOG2L - 4);
  constexpr bool LAST = NS_LOG + RAD_LOG == LOG2L;
  constexpr int TWSH = LOG2L - NS_LOG - RAD_LOG;
#pragma unroll
  for (int i = 0; i < NB; ++i) {
    const int b = t + T * i;
    const int jm = b & (NS - 1);
    V u[RAD];
#pragma unroll
    for (int r = 0; r < RAD; ++r) u[r] = v[i + r * NB];
    if constexpr (NS_LOG > 0) {
#pragma unroll
      for (int r = 1; r < RAD; ++r) {
        V w = team_tw<R, LOG2L>((r * jm) << TWSH, tw);
        if (DIR < 0) w.y = -w.y;
        const V o = u[r];
        u[r] = V{o.x * w.x - o.y * w.y, o.x * w.y + o.y * w.x};
      }
    }
    dft_reg<R, RAD, DIR>(u);
    if constexpr (LAST) {
#pragma unroll
      for (int r = 0; r < RAD; ++r) v[i + r * NB] = u[r];
    } else {
      const int base = ((b - jm) << RAD_LOG) + jm;
#pragma unroll
      for (int r = 0; r < RAD; ++r) xc.put(base + r * NS, u[r]);
    }
  }
  if constexpr (!LAST) {
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kTeamLanes; ++m) v[m] = xc.get(t + T * m);
    __syncthreads();
    team_fft_from<R, DIR, LOG2L, NS_LOG + RAD_LOG, Xch>(v, t, xc, tw);
  }
}

// Unnormalised DFT (DIR = +1: exp(-2 pi i / L) kernel; DIR = -1: its conjugate) of the team's sequence.
// Every lane of the workgroup must call it (it contains workgroup barriers).
template <typename R, int DIR, int LOG2L, class Xch>
__device__ __forceinline__ void team_fft(cx_t<R> (&v)[kTeamLanes], int t, const Xch& xc, const cx_t<R>* tw) {
  static_assert(LOG2L >= 4 && LOG2L <= 12, "team FFT lengths are 16 .. 4096");
  team_fft_from<R, DIR, LOG2L, 0, Xch>(v, t, xc, tw);
}

}  // namespace ldbp
