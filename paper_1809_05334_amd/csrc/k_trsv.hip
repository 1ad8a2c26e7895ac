// Application of the block-diagonal preconditioner of Sec. 2.3 (Eq. 6)
// inside GMRES: z = A_dd^{-1} v for every material domain d, from the LU
// factors of k_lu.hip, by a permutation and blocked forward (L, unit lower)
// and backward (U) substitutions over 512-row diagonal blocks; the inverses
// of the diagonal blocks and the coupling blocks the substitutions use are
// formed once per factorisation.
#include <hip/hip_cooperative_groups.h>
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace vie {

// ------------------------------------------------------------ apply
// z[i] = v[perm[i]] for one block (offset `off` in the global vectors)
__global__ void k_permute(int n, int64_t off, const int32_t *__restrict__ perm, const dz *__restrict__ v,
                          dz *__restrict__ z) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[off + i] = v[off + perm[i]];
}

// Inverses of the kTrsvNB x kTrsvNB diagonal blocks of L (unit lower) and U
// (upper), computed once per factorisation: block b of INV, at b nb^2,
// holds inv(T_bb) row-major with its own size m (nb but for a domain's last
// block) as leading dimension, T_bb the diagonal block at row b*nb.  A
// thread block forms 32 columns of one inverse by substitution; the columns
// live in LDS, and each column's dot products are split over 4 lanes
// (residues of the summation index mod 4, combined by shuffles).  A lane only
// reads back the entries it wrote itself, so no barrier is needed inside the
// substitution.
constexpr int kInvCols = kInvColsH;

template <typename C>
__device__ __forceinline__ void diag_inv_body(const C *__restrict__ F, int64_t ld, int n, int nb, int lower,
                                              C *__restrict__ INV) {
  __shared__ dz X[kInvCols][kTrsvNB];
  const int b = blockIdx.x;
  const int b0 = b * nb;
  const int m = min(nb, n - b0);
  const int cl = threadIdx.x >> 2, t = threadIdx.x & 3;
  const int j = blockIdx.y * kInvCols + cl;      // column of the inverse
  for (int i = t; i < nb; i += 4) X[cl][i] = mk(0, 0);
  const C *T = F + (int64_t)b0 * ld + b0;
  auto inv = [](dz d) {
    const double den = d.re * d.re + d.im * d.im;
    return mk(d.re / den, -d.im / den);
  };
  if (j < m) {
    if (lower) {
      if ((j & 3) == t) X[cl][j] = mk(1, 0);
      for (int i = j + 1; i < m; ++i) {
        const C *Ti = T + (int64_t)i * ld;
        dz s0 = mk(0, 0), s1 = mk(0, 0);
        int l = j + ((t - j) & 3);                 // first l >= j with l = t (mod 4)
        for (; l + 4 < i; l += 8) {
          s0 = s0 + to_dz(Ti[l]) * X[cl][l];
          s1 = s1 + to_dz(Ti[l + 4]) * X[cl][l + 4];
        }
        if (l < i) s0 = s0 + to_dz(Ti[l]) * X[cl][l];
        dz s = s0 + s1;
        s = s + mk(__shfl_xor(s.re, 1), __shfl_xor(s.im, 1));
        s = s + mk(__shfl_xor(s.re, 2), __shfl_xor(s.im, 2));
        if ((i & 3) == t) X[cl][i] = mk(0, 0) - s;
      }
    } else {
      if ((j & 3) == t) X[cl][j] = inv(to_dz(T[(int64_t)j * ld + j]));
      for (int i = j - 1; i >= 0; --i) {
        const C *Ti = T + (int64_t)i * ld;
        dz s0 = mk(0, 0), s1 = mk(0, 0);
        int l = (i + 1) + ((t - (i + 1)) & 3);     // first l > i with l = t (mod 4)
        for (; l + 4 <= j; l += 8) {
          s0 = s0 + to_dz(Ti[l]) * X[cl][l];
          s1 = s1 + to_dz(Ti[l + 4]) * X[cl][l + 4];
        }
        if (l <= j) s0 = s0 + to_dz(Ti[l]) * X[cl][l];
        dz s = s0 + s1;
        s = s + mk(__shfl_xor(s.re, 1), __shfl_xor(s.im, 1));
        s = s + mk(__shfl_xor(s.re, 2), __shfl_xor(s.im, 2));
        if ((i & 3) == t) X[cl][i] = mk(0, 0) - s * inv(to_dz(Ti[i]));
      }
    }
  }
  __syncthreads();
  if (j < m) {
    C *inv_b = INV + (int64_t)b * nb * nb;   // the inverse of block b, m x m row-major: its column j
    for (int i = t; i < m; i += 4) inv_b[(int64_t)i * m + j] = cx<C>::of(X[cl][i]);
  }
}

__global__ __launch_bounds__(4 * kInvCols) void k_diag_inv_z(const dz *F, int64_t ld, int n, int nb, int lower, dz *INV) {
  diag_inv_body(F, ld, n, nb, lower, INV);
}
__global__ __launch_bounds__(4 * kInvCols) void k_diag_inv_c(const fz *F, int64_t ld, int n, int nb, int lower, fz *INV) {
  diag_inv_body(F, ld, n, nb, lower, INV);
}

// Coupling blocks of one domain's sweep: for the matrix blocks b that follow
// another in the sweep's order (b >= 1 for L, b <= nbk - 2 for U), with p =
// b - 1 (L) or b + 1 (U), G_b = T[b, p] inv(T_pp), a kTrsvNB x kTrsvNB
// product in FP64 (rounded to the factor type), written to slot b - 1 (L) or
// b (U) of nb^2 entries, leading dimension nb.  A
// thread block forms a 64 x 64 tile, 4 x 4 entries per thread, through
// 16-deep slices of both operands in shared memory; entries past the blocks'
// sizes are zero.
template <typename C>
__device__ __forceinline__ void coupling_body(const C *__restrict__ F, int64_t ld, int n, int lower,
                                              const C *__restrict__ INV, C *__restrict__ G) {
  constexpr int nb = kTrsvNB, TS = 64, KS = 16;
  __shared__ dz As[TS][KS + 1], Bs[KS][TS + 1];
  const int b = lower ? blockIdx.x + 1 : blockIdx.x;
  const int p = lower ? b - 1 : b + 1;
  const int b0 = b * nb, p0 = p * nb;
  const int mr = min(nb, n - b0), mc = min(nb, n - p0);
  const int tr = blockIdx.y / (nb / TS), tc = blockIdx.y % (nb / TS);
  const int tid = threadIdx.x, ty = tid >> 4, tx = tid & 15;
  const C *__restrict__ Ip = INV + (int64_t)p * nb * nb;   // mc x mc, leading dimension mc
  dz acc[4][4];
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v) acc[u][v] = mk(0, 0);
  for (int k0 = 0; k0 < nb; k0 += KS) {
    // A slice: rows tr*TS .. +TS of T[b, p], columns k0 .. k0+KS; B slice: rows k0 .. of inv(T_pp)
#pragma unroll
    for (int e = tid; e < TS * KS; e += 256) {
      const int rr = e / KS, kk = e % KS;
      const int gr = tr * TS + rr, gk = k0 + kk;
      As[rr][kk] = gr < mr && gk < mc ? to_dz(F[(int64_t)(b0 + gr) * ld + p0 + gk]) : mk(0, 0);
    }
#pragma unroll
    for (int e = tid; e < KS * TS; e += 256) {
      const int kk = e / TS, cc = e % TS;
      const int gk = k0 + kk, gc = tc * TS + cc;
      Bs[kk][cc] = gk < mc && gc < mc ? to_dz(Ip[(int64_t)gk * mc + gc]) : mk(0, 0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < KS; ++kk) {
      dz a[4], bb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) a[u] = As[ty * 4 + u][kk];
#pragma unroll
      for (int v = 0; v < 4; ++v) bb[v] = Bs[kk][tx * 4 + v];
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v) cmac(acc[u][v], a[u], bb[v]);
    }
    __syncthreads();
  }
  C *__restrict__ Gb = G + (int64_t)(lower ? b - 1 : b) * nb * nb;   // slots of the sweep's nbk - 1 blocks
#pragma unroll
  for (int u = 0; u < 4; ++u)
#pragma unroll
    for (int v = 0; v < 4; ++v)
      Gb[(int64_t)(tr * TS + ty * 4 + u) * nb + tc * TS + tx * 4 + v] = cx<C>::of(acc[u][v]);
}
__global__ __launch_bounds__(256) void k_trsv_coupling_z(const dz *F, int64_t ld, int n, int lower, const dz *INV, dz *G) {
  coupling_body(F, ld, n, lower, INV, G);
}
__global__ __launch_bounds__(256) void k_trsv_coupling_c(const fz *F, int64_t ld, int n, int lower, const fz *INV, fz *G) {
  coupling_body(F, ld, n, lower, INV, G);
}

__device__ __forceinline__ dz wave_sum(dz v) {
  for (int o = 32; o > 0; o >>= 1) {
    v.re += __shfl_xor(v.re, o);
    v.im += __shfl_xor(v.im, o);
  }
  return v;
}

// Sums over a 16-lane row of the wave, in every lane of the row, by DPP
// moves (no shared-memory traffic): lane pairs, quads, half rows, rows.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  return __longlong_as_double((long long)dpp64<CTRL>((unsigned long long)__double_as_longlong(v)));
}
__device__ __forceinline__ double row16_sum(double v) {
  v = v + dpp_d<0xb1>(v);    // quad_perm [1,0,3,2]
  v = v + dpp_d<0x4e>(v);    // quad_perm [2,3,0,1]
  v = v + dpp_d<0x141>(v);   // row_half_mirror
  return v + dpp_d<0x140>(v);   // row_mirror
}
__device__ __forceinline__ dz row16_sum(dz v) { return mk(row16_sum(v.re), row16_sum(v.im)); }
// the sum over the whole wave (uniform): the four row sums added in row order
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v = row16_sum(v);
  const auto rl = [](double x, int l) {
    return __longlong_as_double((long long)readlane64((unsigned long long)__double_as_longlong(x), l));
  };
  return ((rl(v, 0) + rl(v, 16)) + rl(v, 32)) + rl(v, 48);
}
__device__ __forceinline__ dz wave_sum_dpp(dz v) { return mk(wave_sum_dpp(v.re), wave_sum_dpp(v.im)); }

// One step of the blocked triangular solves (L forward or U backward) of
// every material domain at once, with nb = kTrsvNB diagonal blocks.  Blocks
// are numbered in the order of the sweep; step j of domain d reduces block j.
// Write r_k = rhs_k - sum over i < k of T[k, i] z_i, so that z_k =
// inv(T_kk) r_k, and precompute per block the coupling G_k = T[k, k-1]
// inv(T_{k-1,k-1}), for which T[k, k-1] z_{k-1} = G_k r_{k-1}.  On entry
//   - z_{j-2}, block [cb0, cb0+cm), is in sol (cm = 0 if j < 2);
//   - r_{j-1} of block [pb0, pb0+pm) is in rin (pm = 0 if j < 1);
//   - for every row of block j, the sum of T[i, k] z_k over the blocks k < j-2
//     is in bsum_in as nci chunk sums (nci = 0 if j < 3).
// The launch has three kinds of work items, numbered in this order:
//   (1) reduction items, 16 rows of block j each:
//       r_j = rhs_j - (its chunk sums) - T[j, j-2] z_{j-2} - G_j r_{j-1},
//       written to rout (the next step's rin);
//   (2) solution items, 16 rows of block j-1 each: z_{j-1} = inv(T_{j-1,j-1})
//       r_{j-1}, written to sol;
//   (3) chunk-sum items: for the rows of block j+1 (if any), the sums of
//       T[i, k] z_k over the blocks k <= j-2 (solutions in sol), columns
//       [bc0, bc0+bk) in chunks of kTrsvSumCols, into bsum_out.
// Only (1) is on the step-to-step chain: one stage of loads, one barrier and
// one dot product per row.  The update reads of (3) run along factor rows,
// so each launch streams whole row segments rather than a strip of one block
// column.  An entry with nm = 0 (the end of a sweep) has only solution items.
// No thread block waits on another; the right-hand sides are only read.
constexpr int kTrsvGroups = kTrsvGroupsH;
constexpr int kTrsvCol = kTrsvNB / 64;   // column chunks of 64 per row

// Loads in these kernels are unconditional, from addresses clamped into the
// domain's arrays, with out-of-range values zeroed afterwards: a load under a
// branch is waited for inside the branch, which would serialise the loads.
__device__ __forceinline__ int clampi(int v, int hi) { return max(0, min(v, hi)); }

// A block-length vector (m entries at src_q, zero past m) of each of NV
// vectors into shared memory.  All threads load (the same addresses
// 1024 / kTrsvNB times over) so that no branch waits for the load before
// the loads that follow are issued; threads below kTrsvNB store.
template <int NV>
struct TrsvVec {
  dz v[NV];
  template <class Src>
  __device__ __forceinline__ void fetch(Src src, int m) {
    const int t = threadIdx.x & (kTrsvNB - 1);
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] = src(q)[clampi(t, m - 1)];
  }
  __device__ __forceinline__ void store(dz *dst, int m) const {   // dst[q * kTrsvNB + t]
    const int t = threadIdx.x;
    if (t >= kTrsvNB) return;
#pragma unroll
    for (int q = 0; q < NV; ++q) dst[q * kTrsvNB + t] = t < m ? v[q] : mk(0, 0);
  }
};

// Shared memory of a step's thread block: reduction and solution items use
// two block-length vectors per right-hand side, chunk-sum items the chunk's
// solutions; one array serves all.
template <int NV, int KC>
struct TrsvLds {
  static constexpr int kChain = 2 * NV * kTrsvNB;
  static constexpr int kChunk = NV * KC;
  static constexpr int kSize = kChain > kChunk ? kChain : kChunk;
};

// KC columns per chunk-sum item (the autotuner picks 1024 or 2048 per
// context; the sums are the same).  NV right-hand sides (1 or 2) share each
// read of the factors; vector q's sums run in the same order for any NV.
template <typename C, int KC, int NV, typename ST = TrsvStep>
__device__ __forceinline__ void trsv_step_body(const ST &st, int vb) {
  static_assert(KC % 1024 == 0, "chunk staging: whole passes of 1024 threads");
  __shared__ dz sm[TrsvLds<NV, KC>::kSize];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // the item's kind and domain: the last entry whose first item of that kind is <= vb
  const int kind = vb < st.chain_blocks ? 0 : (vb < st.z_end ? 1 : 2);
  int d = 0;
  for (int lo = 0, hi = st.ndom - 1; lo <= hi;) {
    const int mid = (lo + hi) >> 1;
    const TrsvDom &M = st.d[mid];
    if ((kind == 0 ? M.first_block : kind == 1 ? M.first_z : M.first_bulk) <= vb) {
      d = mid;
      lo = mid + 1;
    } else {
      hi = mid - 1;
    }
  }
  const TrsvDom &D = st.d[d];
  if (D.active && !*D.active) return;   // (fused batch) a cell whose Arnoldi steps are paused
  const int blk = vb - (kind == 0 ? D.first_block : kind == 1 ? D.first_z : D.first_bulk);
  const int64_t ld = D.ld;
  const C *__restrict__ F = (const C *)D.F;
  if (kind == 0) {
    // (1) row r of block j, one per wave: every load is issued before the
    // barrier (the row's rhs, its entries in block j-2, row r of G_j, its
    // chunk sums, z_{j-2} and r_{j-1} for shared memory)
    const int cb0 = D.cb0, cm = D.cm, pm = D.pm, nb0 = D.nb0, nm = D.nm;
    const int r = 16 * blk + wave;
    const int ic = nb0 + clampi(r, nm - 1);
    dz *zo = sm, *zn = sm + NV * kTrsvNB;
    TrsvVec<NV> po, pn;
    po.fetch([&](int q) { return D.sol[q] + cb0; }, cm);
    pn.fetch([&](int q) { return D.rin + q * kTrsvNB; }, pm);
    dz rv[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) rv[q] = D.rhs[q][ic];
    // (kept in the factor type until used: registers bound the occupancy)
    const int gld = D.gld;
    const C *__restrict__ G = (const C *)D.G + (int64_t)clampi(r, kTrsvNB - 1) * gld;
    C fo[kTrsvCol], fg[kTrsvCol];
#pragma unroll
    for (int c = 0; c < kTrsvCol; ++c) {
      fo[c] = F[(int64_t)ic * ld + cb0 + clampi(lane + 64 * c, cm - 1)];
      fg[c] = G[gld > 0 ? lane + 64 * c : 0];
    }
#pragma unroll
    for (int c = 0; c < kTrsvCol; ++c) {
      if (!(lane + 64 * c < cm)) fo[c] = cx<C>::make(0, 0);
      if (!(lane + 64 * c < pm)) fg[c] = cx<C>::make(0, 0);
    }
    // chunk sums of row r: lane l takes chunks l and l + 64 (bst <= 128; the
    // second only for domains of more than 64 chunks, under a uniform branch)
    dz bs[NV];
    const int bst = D.bst, nci = D.nci;
    const dz *bp = D.bsum_in + (int64_t)clampi(r, kTrsvNB - 1) * bst;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const dz b0 = bp[(int64_t)q * kTrsvNB * bst + clampi(lane, bst - 1)];
      bs[q] = lane < nci ? b0 : mk(0, 0);
    }
    if (nci > 64) {
#pragma unroll
      for (int q = 0; q < NV; ++q) {
        const dz b1 = bp[(int64_t)q * kTrsvNB * bst + clampi(lane + 64, bst - 1)];
        bs[q] = bs[q] + (lane + 64 < nci ? b1 : mk(0, 0));
      }
    }
    po.store(zo, cm);
    pn.store(zn, pm);
    __syncthreads();
    // the chunk sums, then the updates of blocks j-2 and j-1, in that order
    dz rg[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      dz so = mk(0, 0), sn = mk(0, 0);
#pragma unroll
      for (int c = 0; c < kTrsvCol; ++c) cmac(so, to_dz(fo[c]), zo[q * kTrsvNB + lane + 64 * c]);
#pragma unroll
      for (int c = 0; c < kTrsvCol; ++c) cmac(sn, to_dz(fg[c]), zn[q * kTrsvNB + lane + 64 * c]);
      const dz sb = wave_sum_dpp(bs[q]);
      so = wave_sum_dpp(so);
      sn = wave_sum_dpp(sn);
      rg[q] = ((rv[q] - sb) - so) - sn;
    }
    if (lane == 0 && r < nm) {
#pragma unroll
      for (int q = 0; q < NV; ++q) D.rout[q * kTrsvNB + r] = rg[q];
    }
    return;
  }
  if (kind == 1) {
    // (2) row o of inv(T_{j-1,j-1}), one per wave, against r_{j-1}
    const int pb0 = D.pb0, pm = D.pm;
    const int o = 16 * blk + wave;
    dz *zn = sm;
    TrsvVec<NV> pn;
    pn.fetch([&](int q) { return D.rin + q * kTrsvNB; }, pm);
    const C *__restrict__ IV = (const C *)D.INV + (int64_t)clampi(o, pm - 1) * pm;
    C fi[kTrsvCol];
#pragma unroll
    for (int c = 0; c < kTrsvCol; ++c) fi[c] = IV[clampi(lane + 64 * c, pm - 1)];
#pragma unroll
    for (int c = 0; c < kTrsvCol; ++c)
      if (!(lane + 64 * c < pm)) fi[c] = cx<C>::make(0, 0);
    pn.store(zn, pm);
    __syncthreads();
    dz zq[NV];
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      dz a = mk(0, 0);
#pragma unroll
      for (int c = 0; c < kTrsvCol; ++c) cmac(a, to_dz(fi[c]), zn[q * kTrsvNB + lane + 64 * c]);
      zq[q] = wave_sum_dpp(a);
    }
    if (lane == 0 && o < pm) {
#pragma unroll
      for (int q = 0; q < NV; ++q) D.sol[q][pb0 + o] = zq[q];
    }
    return;
  }
  // (a) work item ch of the next block's row group rgp: one row per wave,
  // lane l holding columns l + 64 t of the item's KC columns; the item's
  // solutions are staged in shared memory (zero past the item's end, so
  // clamped factor reads add 0).  Each kTrsvSumCols columns give one chunk
  // sum: lane sums in column order, then the wave sum.
  static_assert(KC % kTrsvSumCols == 0 && kTrsvSumCols == 1024, "chunks of one pass of 1024 threads");
  const int b = blk;
  const int ch = b / D.nrg, rgp = b - ch * D.nrg;
  const int cs = D.bc0 + ch * KC;
  const int cn = min(KC, D.bc0 + D.bk - cs);
  const int sc0 = ch * (KC / kTrsvSumCols);   // the item's first chunk
  const int r = 16 * rgp + wave;
  const int i = D.br0 + clampi(r, D.brm - 1);
  constexpr int kPer = KC / 1024;
  dz zv[NV][kPer];
#pragma unroll
  for (int q = 0; q < NV; ++q)
#pragma unroll
    for (int u = 0; u < kPer; ++u) zv[q][u] = D.sol[q][cs + clampi(tid + 1024 * u, cn - 1)];
  constexpr int T = KC / 64;                                 // factor entries per lane
  constexpr int LB = sizeof(C) == 8 && NV == 1 ? 16 : 8;     // entries per batch of loads
  constexpr int NB = T / LB;
  constexpr int kBatchesPerSum = kTrsvSumCols / 64 / LB;
  static_assert(T % LB == 0 && (kTrsvSumCols / 64) % LB == 0, "whole batches per chunk");
  const C *__restrict__ row = F + (int64_t)i * ld + cs;
  C fa[LB];
#pragma unroll
  for (int u = 0; u < LB; ++u) fa[u] = row[clampi(lane + 64 * u, cn - 1)];
#pragma unroll
  for (int q = 0; q < NV; ++q)
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int t = tid + 1024 * u;
      sm[q * KC + t] = t < cn ? zv[q][u] : mk(0, 0);
    }
  __syncthreads();
  dz s[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) s[q] = mk(0, 0);
  const auto use = [&](const C(&f)[LB], int bt) {
#pragma unroll
    for (int u = 0; u < LB; ++u) {
      const int t = lane + 64 * (bt * LB + u);
      const dz fu = to_dz(f[u]);
#pragma unroll
      for (int q = 0; q < NV; ++q) cmac(s[q], fu, sm[q * KC + t]);
    }
    __builtin_amdgcn_sched_barrier(0);   // no hoisting of one batch's work into another's
  };
  // chunk h of the item done: every vector's wave sum, then lane 0's stores
  // (no vector's arithmetic moves past another's store branch)
  const auto flush = [&](int h) {
#pragma unroll
    for (int q = 0; q < NV; ++q) s[q] = wave_sum_dpp(s[q]);
    if (lane == 0 && r < D.brm && h * kTrsvSumCols < cn) {
#pragma unroll
      for (int q = 0; q < NV; ++q)
        D.bsum_out[(int64_t)q * kTrsvNB * D.bst + (int64_t)r * D.bst + sc0 + h] = s[q];
    }
#pragma unroll
    for (int q = 0; q < NV; ++q) s[q] = mk(0, 0);
  };
  // batch bt + 1 loads while batch bt is used (a rolled loop, so that the
  // compiler keeps two batches in registers rather than hoisting them all);
  // the last batch is used after the loop
#pragma unroll 1
  for (int bt = 0; bt < NB - 1; ++bt) {
    C fb[LB];
#pragma unroll
    for (int u = 0; u < LB; ++u) fb[u] = row[clampi(lane + 64 * ((bt + 1) * LB + u), cn - 1)];
    use(fa, bt);
    if ((bt + 1) % kBatchesPerSum == 0) flush(bt / kBatchesPerSum);
#pragma unroll
    for (int u = 0; u < LB; ++u) fa[u] = fb[u];
  }
  use(fa, NB - 1);
  flush(KC / kTrsvSumCols - 1);
}

#define VIE_TRSV_STEP(T, C, K)                                                                  \
  __global__ __launch_bounds__(1024) void k_trsv_step_##T##_k##K(TrsvStep st) {                \
    trsv_step_body<C, K, 1>(st, blockIdx.x);                                                  \
  }                                                                                           \
  __global__ __launch_bounds__(1024) void k_trsv_step2_##T##_k##K(TrsvStep st) {               \
    trsv_step_body<C, K, 2>(st, blockIdx.x);                                                  \
  }
VIE_TRSV_STEP(z, dz, 1024)
VIE_TRSV_STEP(z, dz, 2048)
VIE_TRSV_STEP(c, fz, 1024)
VIE_TRSV_STEP(c, fz, 2048)

// Every step of the triangular solves in one cooperative launch: the thread
// blocks share each step's work items (the same items the per-step launches
// give to their thread blocks) and meet at a grid barrier between steps,
// which orders one step's partial products before the next step's sums.
// All blocks run the same loops and reach every barrier.
template <typename C, int KC>
__device__ __forceinline__ void trsv_coop_body(const TrsvStep *__restrict__ plan, int nsteps) {
  cooperative_groups::grid_group grid = cooperative_groups::this_grid();
  for (int s = 0; s < nsteps; ++s) {
    const TrsvStep &st = plan[s];
    const int total = st.total_blocks;
    for (int vb = blockIdx.x; vb < total; vb += gridDim.x) {
      __syncthreads();   // the previous item's shared memory is free
      trsv_step_body<C, KC, 1>(st, vb);
    }
    grid.sync();
  }
}

// One step of a batch's fused triangular solves (one vector per cell): the
// step's domains of every cell, read from device memory.
struct TrsvStepDev {
  const TrsvDom *d;
  int ndom, lower, chain_blocks, z_end;
};
#define VIE_TRSV_STEPD(T, C)                                                                      \
  __global__ __launch_bounds__(1024) void k_trsv_stepd_##T(const TrsvDom *doms, int ndom, int lower,   \
                                                            int chain_blocks, int z_end) {             \
    const TrsvStepDev st{doms, ndom, lower, chain_blocks, z_end};                                     \
    trsv_step_body<C, kTrsvSumCols, 1, TrsvStepDev>(st, blockIdx.x);                             \
  }
VIE_TRSV_STEPD(z, dz)
VIE_TRSV_STEPD(c, fz)

#define VIE_TRSV_COOP(T, C, K)                                                                  \
  __global__ __launch_bounds__(1024) void k_trsv_coop_##T##_k##K(const TrsvStep *plan, int nsteps) { \
    trsv_coop_body<C, K>(plan, nsteps);                                                       \
  }
VIE_TRSV_COOP(z, dz, 1024)
VIE_TRSV_COOP(z, dz, 2048)
VIE_TRSV_COOP(c, fz, 1024)
VIE_TRSV_COOP(c, fz, 2048)

}  // namespace vie
