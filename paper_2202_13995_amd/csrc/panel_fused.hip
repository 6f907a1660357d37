// One-launch panel factorization.
//
// Paper, section "High Performance Linpack", "Base Implementation": each
// iteration first decomposes the diagonal block (the LU kernel) and updates the
// blocks below it (the left blocks).  With partial pivoting these form one tall
// column panel, factored here by a single persistent launch so that, while the
// previous iteration's inner-block multiplication occupies the GPU, the panel
// waits for compute units once instead of once per sub-step.
//
// G workgroups (at most one per compute unit, all resident) split the panel's
// rows [c0, m) into consecutive blocks of R rows (R a multiple of 32).  The
// panel's W columns are processed right-looking in leaves of 32 columns:
//   (A) each workgroup loads its rows of the leaf into LDS (column-major);
//   (B) per column: every workgroup publishes its best candidate (largest |a|,
//       lowest row on ties, NaN below every number), all meet at a grid
//       barrier, every workgroup picks the same winner, exchanges the pivot
//       and diagonal rows inside the leaf, scales by the pivot (division) and
//       applies the rank-1 update to the rest of the leaf;
//   (C) the factored leaf is written back;
//   (D) the leaf's row exchanges are applied to the panel's other columns:
//       each workgroup copies, for every destination row it owns, the source
//       row to a staging buffer; grid barrier; then copies staging to the
//       destination (the net permutation of the leaf's swaps comes from the
//       same parallel plan as the full-matrix exchanges);
//   (E) the workgroup owning the leaf's rows solves them against the leaf's
//       unit lower triangle (the "top" update inside the panel); grid barrier;
//   (F) every workgroup subtracts L(own rows, leaf) * U(leaf rows, right of the
//       leaf) from its rows below the leaf on the matrix cores.
// All data one workgroup writes and another reads moves through relaxed
// agent-scope atomics (L2-coherent accesses), so no fence ever writes back or
// invalidates the L2 (see grid_barrier).
#include <climits>
#include <type_traits>

#include "common.h"
#include "device.h"
#include "swap_plan.h"

namespace lp {
namespace {

constexpr int kLW = 32;          // the widest leaf (leaf width LW is 16 or 32)
constexpr int kChunk = 256;      // rows per thread-sweep (one per thread); RPT chunks per workgroup
constexpr int kMaxEnt = 2 * kLW;  // gather entries of one leaf's exchanges
constexpr int kLd = 8;            // leaf-load elements in flight per thread
constexpr int kXb = 8;            // exchange elements in flight per thread (binary32; 4 for binary64)
constexpr int kMaxG = 256;        // workgroups per panel launch
// one key per (column, workgroup), workgroup-major with a padded stride so
// that the keys of one column, which every workgroup polls, fall on many
// memory channels
constexpr int kKeyStride = 1024 + 32;
constexpr int kKeySlots = kKeyStride * kMaxG;

// Calls f(std::integral_constant<int, J>) for J = J0 .. N-1 in order while it
// returns true; the index is a compile-time constant inside f.
template <int J, int N, typename F>
__device__ __forceinline__ bool static_for(F& f) {
  if constexpr (J < N) {
    if (!f(std::integral_constant<int, J>{})) return false;
    return static_for<J + 1, N>(f);
  } else {
    return true;
  }
}

__device__ __forceinline__ void wg_sync() {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
}

template <typename T, int RPT, int LW>
__global__ __launch_bounds__(256, (RPT == 1) ? 2 : 1) void panel_fused_kernel(
    int m, int c0, int W, T* __restrict__ A, long long lda, int32_t* __restrict__ ipiv,
    int32_t* __restrict__ info, int R, int G, char* __restrict__ slots,
    unsigned* __restrict__ barrier, T* __restrict__ staging,
    unsigned long long* __restrict__ keys, unsigned long long* __restrict__ keys_next,
    int nopiv, int CW) {
  typedef Mfma16<T> MF;
  typedef typename MF::acc acc_t;
  // row blocks of 16 per load batch in (F) (8 for binary64: more were slower)
  constexpr int kRbb = (sizeof(T) == 8) ? 8 : 16;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  // [RPT][LW][kChunk]: one row chunk column-major while loading and writing
  // the leaf, all of the workgroup's rows during (F)
  T* stage = reinterpret_cast<T*>(smem_raw);
  __shared__ T lblk[kLW * (kLW + 1)];         // the leaf's own rows (diagonal block), row-major
  __shared__ double red_key[2][4];
  __shared__ int red_idx[2][4];
  __shared__ T wrow[2][4][kLW];  // each wave's candidate row, by column parity
  __shared__ T drw[2][kLW];      // the diagonal row, by column parity
  __shared__ T prow[kLW];
  __shared__ T drow[kLW];
  __shared__ int s_flag;
  __shared__ int s_piv[kLW];
  __shared__ int pl_nxt[kLW];
  __shared__ int pl_B[kLW];
  __shared__ int pl_flag[2 * kLW];
  __shared__ int pl_dst[kMaxEnt];
  __shared__ int pl_src[kMaxEnt];
  __shared__ int pl_n;
  __shared__ int pl_own[kMaxEnt];
  __shared__ int pl_nown;
  __shared__ unsigned long long red_enc[4];
  __shared__ int red_g[4];
  __shared__ int s_timeout;
  __shared__ int s_pw;
  __shared__ int s_dflag;

  const LeafLayout lay = leaf_layout(G);
  const int g = blockIdx.x;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int base = c0 + g * R;
  const int nrows = min(R, m - base);
  unsigned nbar = 0;
  // the first zero pivot so far (read once; only this launch writes it meanwhile)
  int info_val = (g == 0 && tid == 0) ? *info : 0;
  // the next panel launch has at most CW columns; it may have more
  // workgroups than this one, so every key slot of those columns is cleared
  if (G > 1) {  // a single-workgroup launch is followed by single-workgroup launches
    for (int e = g * blockDim.x + tid; e < CW * kMaxG; e += G * blockDim.x)
      xstore(&keys_next[(size_t)(e / CW) * kKeyStride + e % CW], 0ull);
  }
  // the panel is the critical path while the trailing update runs beside it
  // on the same compute units: its waves issue first
  __builtin_amdgcn_s_setprio(3);
  if (tid == 0) s_timeout = 0;

  // every workgroup executes the same sequence of these
  auto sync_all = [&]() -> bool {
    if (G == 1) {
      wg_sync();
      return true;
    }
    const bool ok = grid_barrier(barrier, (unsigned)G * (nbar + 1u), &s_flag);
    ++nbar;
    return ok;
  };

  const int nleaf = (W + LW - 1) / LW;
  for (int b = 0; b < nleaf; ++b) {
    const int cb = c0 + b * LW;
    const int wb = min(LW, c0 + W - cb);
    const int right0 = cb + wb;
    const int nright = c0 + W - right0;
    const int rlo = max(cb - base, 0);

    // (A) the leaf's rows >= cb, in chunks of 256 rows: coalesced loads into
    // LDS, then each thread takes its row of the chunk into registers
    T x[RPT][LW];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r0 = kChunk * q;
      const int lo = max(rlo, r0), hi = min(nrows, r0 + kChunk);
      // kLd loads in flight per thread; out-of-range slots load a valid
      // element and drop it (a load under a branch would wait in the branch)
      const int e_lo = (lo - r0) * wb, e_hi = (hi - r0) * wb;
      for (int e0 = e_lo + tid; e0 < e_hi; e0 += kLd * 256) {
        T v[kLd];
#pragma unroll
        for (int u = 0; u < kLd; ++u) {
          const int e = min(e0 + u * 256, e_hi - 1);
          const int r = e / wb;
          v[u] = xload(&A[(long long)(base + r0 + r) * lda + cb + (e - r * wb)]);
        }
#pragma unroll
        for (int u = 0; u < kLd; ++u) {
          const int e = e0 + u * 256;
          if (e < e_hi) {
            const int r = e / wb;
            stage[(e - r * wb) * kChunk + r] = v[u];
          }
        }
      }
      __syncthreads();
      const int r = r0 + tid;
      const bool act = r >= rlo && r < nrows;
#pragma unroll
      for (int c = 0; c < LW; ++c) x[q][c] = (act && c < wb) ? stage[c * kChunk + tid] : T(0);
      __syncthreads();
    }

    // (B) the leaf's columns; the column index is a compile-time constant in
    // every step so that the rows stay in registers
    auto column = [&](auto jc) -> bool {
      constexpr int jj = decltype(jc)::value;
      if (jj < wb) {
        const int dg = cb + jj;
        const int par = jj & 1;
        double bk = -2.0;
        int bi = INT_MAX;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const int r = tid + 256 * q;
          const int gi = base + r;
          if (!nopiv && r < nrows && gi >= dg) {
            const T v = x[q][jj];
            const double k = (v != v) ? -1.0 : fabs((double)v);
            if (better(k, gi, bk, bi)) {
              bk = k;
              bi = gi;
            }
          }
        }
        {
          unsigned long long kb = (unsigned long long)__double_as_longlong(bk);
          wave_best(kb, bi, [](unsigned long long ka, int ia, unsigned long long kc, int ic) {
            return better(__longlong_as_double((long long)ka), ia,
                          __longlong_as_double((long long)kc), ic);
          });
          bk = __longlong_as_double((long long)kb);
        }
        // the wave's candidate row and the diagonal row go to LDS
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const int gi = base + tid + 256 * q;
          if (bi != INT_MAX && gi == bi) {
#pragma unroll
            for (int c = 0; c < LW; ++c) wrow[par][wave][c] = x[q][c];
          }
          if (gi == dg && tid + 256 * q < nrows) {
#pragma unroll
            for (int c = 0; c < LW; ++c) drw[par][c] = x[q][c];
          }
        }
        if (lane == 0) {
          red_key[par][wave] = bk;
          red_idx[par][wave] = bi;
        }
        __syncthreads();
        int wbest = 0;
        bk = red_key[par][0];
        bi = red_idx[par][0];
#pragma unroll
        for (int t = 1; t < 4; ++t)
          if (better(red_key[par][t], red_idx[par][t], bk, bi)) {
            bk = red_key[par][t];
            bi = red_idx[par][t];
            wbest = t;
          }
        const bool own_diag = dg >= base && dg < base + nrows;
        int p;
        const T* urow;  // the pivot row (LDS)
        const T* drv;   // the old diagonal row (LDS)
        if (G == 1) {
          // without pivoting (nopiv) the diagonal row is the pivot row
          const T dv = drw[par][jj];
          p = (nopiv || dv != dv) ? dg : bi;
          drv = drw[par];
          urow = (p == dg) ? drv : wrow[par][wbest];
        } else {
          // publish the candidate row and index (and, from the owner, the
          // diagonal row and its NaN flag) as tagged words, then the key; a
          // non-zero key says this workgroup reached the column, the tags say
          // which words have landed
          char* sb = slots + (size_t)par * lay.buf_bytes;
          unsigned long long* recs = reinterpret_cast<unsigned long long*>(sb + lay.rec_off);
          unsigned long long* drec = reinterpret_cast<unsigned long long*>(sb + lay.drec_off);
          unsigned long long* ckeys = keys + (size_t)(dg - c0);  // stride kKeyStride
          constexpr int kWPV = (int)(sizeof(T) / 4);  // 32-bit words per value
          constexpr int kIdxW = 2 * kLeafMax;         // index / flag word
          const int nw = kWPV * wb;
          const unsigned tag = (unsigned)(dg + 1);
          unsigned long long* myrec = recs + (size_t)g * kRecWords;
          if (tid < nw && bi != INT_MAX)
            xstore(&myrec[tid],
                   tagged(tag, reinterpret_cast<const unsigned*>(wrow[par][wbest])[tid]));
          if (tid == kIdxW) xstore(&myrec[kIdxW], tagged(tag, (unsigned)bi));
          if (own_diag) {
            if (tid >= 128 && tid < 128 + nw)
              xstore(&drec[tid - 128],
                     tagged(tag, reinterpret_cast<const unsigned*>(drw[par])[tid - 128]));
            if (tid == 128 + kIdxW) {
              const T dv = drw[par][jj];
              xstore(&drec[kIdxW], tagged(tag, (dv != dv) ? 1u : 0u));
            }
          }
          if (tid == 0) {
            unsigned long long ek = 1ull;  // no candidate
            if (bi != INT_MAX)
              ek = (bk < 0.0) ? 2ull : 3ull + (unsigned long long)__double_as_longlong(bk);
            xstore(&ckeys[(size_t)g * kKeyStride], ek);
          }
          // wait for every workgroup's key; the largest wins, the lowest
          // workgroup (hence the lowest row) on ties
          unsigned long long kv = 0ull;
          int kg = INT_MAX;
          if (tid < G) {
            const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
            while ((kv = xload(&ckeys[(size_t)tid * kKeyStride])) == 0ull) {
              __builtin_amdgcn_s_sleep(1);
              if (__builtin_amdgcn_s_memrealtime() - t0 > kBarrierTimeoutTicks) {
                s_timeout = 1;
                break;
              }
            }
            kg = tid;
          }
          wave_best(kv, kg, [](unsigned long long a, int ia, unsigned long long b, int ib) {
            return a > b || (a == b && ia < ib);
          });
          if (lane == 0) {
            red_enc[wave] = kv;
            red_g[wave] = kg;
          }
          __syncthreads();
          if (s_timeout) {
            if (g == 0 && tid == 0) *info = LP_INFO_BARRIER_TIMEOUT;
            return false;
          }
          kv = red_enc[0];
          kg = red_g[0];
#pragma unroll
          for (int t = 1; t < 4; ++t)
            if (red_enc[t] > kv || (red_enc[t] == kv && red_g[t] < kg)) {
              kv = red_enc[t];
              kg = red_g[t];
            }
          // the winner's row and index, the diagonal row and its flag: read
          // until every word carries this column's tag
          {
            const unsigned long long* wrec = recs + (size_t)kg * kRecWords;
            unsigned* pbuf = reinterpret_cast<unsigned*>(prow);
            unsigned* dbuf = reinterpret_cast<unsigned*>(drow);
            const unsigned long long t0 = __builtin_amdgcn_s_memrealtime();
            for (;;) {
              int bad = 0;
              if (tid < nw) {
                const unsigned long long w = xload(&wrec[tid]);
                bad = (unsigned)(w >> 32) != tag;
                pbuf[tid] = (unsigned)w;
              } else if (tid == kIdxW) {
                const unsigned long long w = xload(&wrec[kIdxW]);
                bad = (unsigned)(w >> 32) != tag;
                s_pw = (int)(unsigned)w;
              } else if (tid >= 128 && tid < 128 + nw) {
                const unsigned long long w = xload(&drec[tid - 128]);
                bad = (unsigned)(w >> 32) != tag;
                dbuf[tid - 128] = (unsigned)w;
              } else if (tid == 128 + kIdxW) {
                const unsigned long long w = xload(&drec[kIdxW]);
                bad = (unsigned)(w >> 32) != tag;
                s_dflag = (int)(unsigned)w;
              }
              if (!__syncthreads_or(bad)) break;
              if (tid == 0 && __builtin_amdgcn_s_memrealtime() - t0 > kBarrierTimeoutTicks)
                s_timeout = 1;
              __syncthreads();
              if (s_timeout) {
                if (g == 0 && tid == 0) *info = LP_INFO_BARRIER_TIMEOUT;
                return false;
              }
              __builtin_amdgcn_s_sleep(1);
            }
          }
          p = s_dflag ? dg : s_pw;
          drv = drow;
          urow = (p == dg) ? drv : prow;
        }
        const T piv = urow[jj];
        if (tid == 0) s_piv[jj] = p;
        if (g == 0 && tid == 0) {
          ipiv[dg] = p;
          if (piv == T(0) && info_val == 0) {
            info_val = dg + 1;
            *info = info_val;
          }
        }
        // exchange rows dg and p, then scale and update the rows below
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
          const int r = tid + 256 * q;
          const int gi = base + r;
          if (p != dg && r < nrows) {
            if (gi == p) {
#pragma unroll
              for (int c = 0; c < LW; ++c) x[q][c] = drv[c];
            } else if (gi == dg) {
#pragma unroll
              for (int c = 0; c < LW; ++c) x[q][c] = urow[c];
            }
          }
          if (piv != T(0) && r < nrows && gi > dg) {
            const T l = x[q][jj] / piv;
            x[q][jj] = l;
#pragma unroll
            for (int c = jj + 1; c < LW; ++c) x[q][c] -= l * urow[c];
          }
        }
        if (G > 1) __syncthreads();  // prow/drow/s_pw/s_dflag are reused by the next column
      }
      return true;
    };
    if (!static_for<0, LW>(column)) return;

    // (C) the factored leaf back to memory in chunks of 256 rows (coalesced
    // through LDS); the leaf's own rows also go to lblk for the solve in (E)
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
      const int r0 = kChunk * q;
      const int r = r0 + tid;
      if (r >= rlo && r < nrows) {
#pragma unroll
        for (int c = 0; c < LW; ++c)
          if (c < wb) stage[c * kChunk + tid] = x[q][c];
      }
      const int li = r - (cb - base);
      if (li >= 0 && li < wb) {
#pragma unroll
        for (int c = 0; c < LW; ++c) lblk[li * (kLW + 1) + c] = x[q][c];
      }
      __syncthreads();
      const int lo = max(rlo, r0), hi = min(nrows, r0 + kChunk);
      for (int e = (lo - r0) * wb + tid; e < (hi - r0) * wb; e += blockDim.x) {
        const int rr = e / wb;
        const int c = e - rr * wb;
        xstore(&A[(long long)(base + r0 + rr) * lda + cb + c], stage[c * kChunk + rr]);
      }
      __syncthreads();
    }

    // (D) the leaf's exchanges on the panel's other columns
    build_swap_plan(s_piv, cb, cb + wb, pl_nxt, pl_B, nullptr, pl_flag, pl_dst, pl_src, &pl_n);
    __syncthreads();
    const int nent = pl_n;
    const int nout = W - wb;
    const int nleft = cb - c0;
    if (nout > 0 && nent > 0) {
      // this workgroup's destinations, compacted by the first wave
      if (wave == 0) {
        const bool own = lane < nent && (pl_dst[lane] - c0) / R == g;
        const unsigned long long mask = __ballot(own);
        if (own) pl_own[__popcll(mask & ((1ull << lane) - 1ull))] = lane;
        if (lane == 0) pl_nown = __popcll(mask);
      }
      __syncthreads();
      const int tot = pl_nown * nout;
      // every load of a round is issued before its stores: one fabric round
      // trip per kXb elements per thread
      auto move = [&](bool gather) {
        constexpr int XB = sizeof(T) == 4 ? kXb : kXb / 2;
        for (int e0 = tid; e0 < tot; e0 += XB * 256) {
          T v[XB];
#pragma unroll
          for (int u = 0; u < XB; ++u) {
            const int e2 = min(e0 + u * 256, tot - 1);
            const int e = pl_own[e2 / nout];
            const int ci = e2 % nout;
            const int col = (ci < nleft) ? c0 + ci : ci + wb + c0;
            v[u] = gather ? xload(&A[(long long)pl_src[e] * lda + col])
                          : xload(&staging[(long long)e * W + ci]);
          }
#pragma unroll
          for (int u = 0; u < XB; ++u) {
            const int e2 = e0 + u * 256;
            if (e2 < tot) {
              const int e = pl_own[e2 / nout];
              const int ci = e2 % nout;
              const int col = (ci < nleft) ? c0 + ci : ci + wb + c0;
              if (gather)
                xstore(&staging[(long long)e * W + ci], v[u]);
              else
                xstore(&A[(long long)pl_dst[e] * lda + col], v[u]);
            }
          }
        }
      };
      move(true);
      if (!sync_all()) {
        if (g == 0 && tid == 0) *info = LP_INFO_BARRIER_TIMEOUT;
        return;
      }
      move(false);
    }
    if (nright <= 0) {
      wg_sync();
      continue;
    }

    // (E) the leaf's rows right of the leaf: U = L_bb^-1 * A(leaf rows, right)
    if ((cb - c0) / R == g) {
      wg_sync();
      for (int col = tid; col < nright; col += blockDim.x) {
        T x[LW];
#pragma unroll
        for (int i = 0; i < LW; ++i)
          x[i] = xload(&A[(long long)(cb + min(i, wb - 1)) * lda + right0 + col]);
#pragma unroll
        for (int i = 0; i < LW; ++i)
          if (i >= wb) x[i] = T(0);
#pragma unroll
        for (int i = 1; i < LW; ++i) {
          if (i < wb) {
            T acc = x[i];
#pragma unroll
            for (int k = 0; k < i; ++k) acc -= lblk[i * (kLW + 1) + k] * x[k];
            x[i] = acc;
          }
        }
#pragma unroll
        for (int i = 0; i < LW; ++i)
          if (i < wb) xstore(&A[(long long)(cb + i) * lda + right0 + col], x[i]);
      }
    }
    if (!sync_all()) {
      if (g == 0 && tid == 0) *info = LP_INFO_BARRIER_TIMEOUT;
      return;
    }

    // (F) own rows below the leaf: A(r, right) -= L(r, leaf) * U(leaf, right).
    // The L values of all the workgroup's rows go to LDS first, so the leaf's
    // registers are free and each wave keeps kRbb row blocks of loads in
    // flight over the whole row range; every row block of one 16-column block
    // reuses the U values loaded once.
    const int r_first = max(right0 - base, 0);
    if (r_first < nrows) {  // the same for the whole workgroup
      const int gq = lane >> 4;
      const int l16 = lane & 15;
      const int ncb = (nright + 15) >> 4;
#pragma unroll
      for (int q = 0; q < RPT; ++q)
#pragma unroll
        for (int c = 0; c < LW; ++c) stage[(q * LW + c) * kChunk + tid] = x[q][c];
      __syncthreads();
      const int rb0 = r_first & ~15;
      const int nrb = (nrows - rb0 + 15) >> 4;
      for (int cbk = wave; cbk < ncb; cbk += 4) {
        const int col = right0 + 16 * cbk + l16;
        const bool colok = col < c0 + W;
        T bfr[LW / 16][4];
#pragma unroll
        for (int s2 = 0; s2 < LW / 16; ++s2)
#pragma unroll
          for (int t = 0; t < 4; ++t) {
            const int k = 16 * s2 + MF::kidx(gq, t);
            const bool ok = k < wb && colok;
            const T raw = xload(&A[ok ? (long long)(cb + k) * lda + col : (long long)cb * lda + c0]);
            bfr[s2][t] = ok ? raw : T(0);
          }
        // all row blocks of a batch are loaded before the first product, so a
        // batch costs one round trip to memory
        for (int rg = 0; rg < nrb; rg += kRbb) {
          acc_t acc[kRbb];
#pragma unroll
          for (int u = 0; u < kRbb; ++u) {
            const int rloc = rb0 + 16 * (rg + u);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int row = rloc + MF::drow(gq, v);
              const bool ok = (rg + u < nrb) && row >= r_first && row < nrows && colok;
              const T raw =
                  xload(&A[ok ? (long long)(base + row) * lda + col : (long long)base * lda + c0]);
              acc[u][v] = ok ? -raw : T(0);
            }
          }
#pragma unroll
          for (int u = 0; u < kRbb; ++u) {
            if (rg + u >= nrb) continue;
            // the row block's L values first (rows past nrows hold zeros),
            // then its products
            const int arow = rb0 + 16 * (rg + u) + l16;  // < RPT * kChunk
            const int sq = arow >> 8, sr = arow & (kChunk - 1);
            T av[LW / 16][4];
#pragma unroll
            for (int s2 = 0; s2 < LW / 16; ++s2)
#pragma unroll
              for (int t = 0; t < 4; ++t) {
                const int k = 16 * s2 + MF::kidx(gq, t);
                const bool ok = k < wb;
                const T a0 = stage[ok ? (sq * LW + k) * kChunk + sr : 0];
                av[s2][t] = ok ? a0 : T(0);
              }
#pragma unroll
            for (int s2 = 0; s2 < LW / 16; ++s2)
#pragma unroll
              for (int t = 0; t < 4; ++t) acc[u] = MF::mma(av[s2][t], bfr[s2][t], acc[u]);
          }
#pragma unroll
          for (int u = 0; u < kRbb; ++u) {
            const int rloc = rb0 + 16 * (rg + u);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
              const int row = rloc + MF::drow(gq, v);
              const bool ok = (rg + u < nrb) && row >= r_first && row < nrows && colok;
              if (ok) xstore(&A[(long long)(base + row) * lda + col], -acc[u][v]);
            }
          }
        }
      }
      __syncthreads();
    }
    wg_sync();
  }
}

}  // namespace

size_t panel_staging_bytes(int W) { return sizeof(double) * (size_t)kMaxEnt * (size_t)W; }
size_t panel_keys_bytes() { return sizeof(unsigned long long) * (size_t)kKeySlots; }

template <typename T>
int launch_panel_fused(int m, int c0, int W, T* A, long long lda, int32_t* ipiv, int32_t* info,
                       void* slots, unsigned* barrier, void* staging, void* keys,
                       void* keys_next, hipStream_t s, int max_wgs, bool nopiv, int next_w) {
  const int rows = m - c0;
  const int CW = std::max(W, next_w);
  if (rows <= 0 || W <= 0) return LP_OK;
  if (W > rows) return LP_ENOTSUP;
  if (nopiv && rows > kPanelRowsPerWg) return LP_ENOTSUP;  // one workgroup only
  const int ncu = num_cus();
  int R, G;
  if (rows <= kPanelRowsPerWg) {
    R = (rows + 31) & ~31;  // one workgroup: no cross-workgroup exchange
    G = 1;
  } else if (max_wgs > 0) {
    // a reserved set of compute units: as few workgroups as cover the rows
    R = (int)cdiv(rows, max_wgs);
    R = (R + 31) & ~31;
    if (R < kChunk) R = kChunk;
    if (R > kPanelRowsPerWg) return LP_ENOTSUP;
    G = (int)cdiv(rows, R);
  } else {
    // the whole chip: many small workgroups
    R = (int)cdiv(rows, std::min(ncu, 256));
    R = (R + 31) & ~31;
    if (R < kChunk) R = kChunk;
    G = (int)cdiv(rows, R);
  }
  if (R > kPanelRowsPerWg || G > ncu || G > kMaxG || CW > 1024) return LP_ENOTSUP;
  // 1024 binary64 rows per workgroup keep 16-wide leaves in registers
#define LP_PANEL_LAUNCH(RPTV, LWV)                                                               \
  hipLaunchKernelGGL((panel_fused_kernel<T, RPTV, LWV>), dim3(G), dim3(256),                     \
                     sizeof(T) * (size_t)kChunk * (LWV) * (RPTV), s, m, c0, W, A,                \
                     lda,                                                                        \
                     ipiv, info, R, G, (char*)slots, barrier, (T*)staging,                       \
                     (unsigned long long*)keys, (unsigned long long*)keys_next, nopiv ? 1 : 0,  \
                     CW)
  if (R <= kChunk)
    LP_PANEL_LAUNCH(1, 32);
  else if (R <= 2 * kChunk)
    LP_PANEL_LAUNCH(2, 32);
  else if constexpr (sizeof(T) == 8)
    LP_PANEL_LAUNCH(4, 16);
  else
    LP_PANEL_LAUNCH(4, 32);
#undef LP_PANEL_LAUNCH
  LP_LAUNCH_CHECK();
  return LP_OK;
}

template int launch_panel_fused<double>(int, int, int, double*, long long, int32_t*, int32_t*,
                                        void*, unsigned*, void*, void*, void*, hipStream_t, int,
                                        bool, int);
template int launch_panel_fused<float>(int, int, int, float*, long long, int32_t*, int32_t*,
                                       void*, unsigned*, void*, void*, void*, hipStream_t, int,
                                       bool, int);

}  // namespace lp
