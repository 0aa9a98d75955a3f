// tsne_symmetrize: P = (C + C^T) / (2n) on the union of the kNN patterns
// (van der Maaten & Hinton 2008, Sec. 3.1; sparse pattern as in van der
// Maaten 2014, Sec. 4.1), as CSR with ascending columns plus the transpose
// positions.  HBM-bound integer work, deterministic:
//   1. the transposed lists: a stable radix sort (radix.hpp) of the directed
//      entries e = i k + t by their target j, so each target's list holds
//      its sources in ascending order (the entries are numbered in source
//      order); invalid targets sort to a bucket n of their own and are
//      reported through err
//   2. in_ptr from the sorted targets (each boundary writes the starts of
//      the targets it passes), then the sources e / k and values p_e of the
//      lists, with a repeated (j, i) reported through err
//   3. (steps 1-2 replace an in-degree histogram, an atomic scatter and a
//      per-list sort, which took 22 of 28 ms at 10^6 points, k = 90)
//   4. sort each row's k out-entries by column (wave bitonic sort)
//   5. union size per row (binary search of each out-entry in the in-list),
//      scan -> row_ptr
//   6. merge by ranks: position of an element = its rank in its own list +
//      its rank in the other list - the shared entries before it
//   7. tpos by binary search of i in row col[e]
// Entry values are (p_{j|i} + p_{i|j}) / (2n) in row i and
// (p_{i|j} + p_{j|i}) / (2n) in row j: the same FP32 sum, so P = P^T bitwise.
// tsne_umap_fuzzy_union runs the same steps with the probabilistic t-conorm
// b = (a + a') - a a' of the two directed weights in step 6 (McInnes, Healy &
// Melville 2018, Sec. 3.1), symmetric bitwise for the same reason.
#include "common.hpp"
#include "radix.hpp"
#include "scan.hpp"

namespace tsne {

__device__ __forceinline__ bool edge_ok(int64_t i, int32_t j, int64_t n) { return j >= 0 && j < n && j != i; }

// Sort key of directed entry e = (i, j = nbr[e]): its target, or n for an
// invalid target (out of range or i itself), which is reported.
__global__ __launch_bounds__(256) void sym_keys_kernel(const int32_t* __restrict__ nbr, int64_t n, int k,
                                                       int32_t* __restrict__ key, int32_t* __restrict__ ent,
                                                       int* __restrict__ err) {
  const int64_t e = gtid();
  if (e >= n * k) return;
  const int64_t i = e / k;
  const int32_t j = nbr[e];
  const bool ok = edge_ok(i, j, n);
  if (!ok) atomicOr(err, 1);
  key[e] = ok ? j : int32_t(n);
  ent[e] = int32_t(e);
}

// in_ptr[j] = first position of target j in the sorted keys, j = 0 .. n
// (in_ptr[n] = the number of valid entries): position p writes the starts
// of the targets after key[p - 1] up to key[p].
__global__ __launch_bounds__(256) void sym_inptr_kernel(const int32_t* __restrict__ skey, int64_t nk, int64_t n,
                                                        int64_t* __restrict__ in_ptr) {
  const int64_t p = gtid();
  if (p > nk) return;
  const int64_t prev = p > 0 ? int64_t(skey[p - 1]) : -1;
  const int64_t cur = p < nk ? int64_t(skey[p]) : n + 1;
  const int64_t hi = cur < n ? cur : n;
  for (int64_t j = prev + 1; j <= hi; ++j) in_ptr[j] = p;
}

// Sources and values of the transposed lists; a source repeated within one
// list (a row that names the same neighbour twice) is reported.
__global__ __launch_bounds__(256) void sym_lists_kernel(const int32_t* __restrict__ skey,
                                                        const int32_t* __restrict__ sent,
                                                        const float* __restrict__ Pc, const int64_t* __restrict__ in_ptr,
                                                        int64_t n, int k, int32_t* __restrict__ s_src,
                                                        float* __restrict__ s_val, int* __restrict__ err) {
  const int64_t p = gtid();
  if (p >= in_ptr[n]) return;
  const int32_t e = sent[p];
  const int32_t i = e / k;
  s_src[p] = i;
  s_val[p] = Pc[e];
  if (p > 0 && skey[p - 1] == skey[p] && sent[p - 1] / k == i) atomicOr(err, 1);
}

// Sort of one list of at most EPL*64 (index, value) entries by one wave
// (register bitonic sort of index << 32 | value bits).  Indices in one list
// are distinct for valid input, so the order is by index; a repeated index
// (invalid input) is reported through err.
template <int EPL>
__device__ void wave_bitonic_segment(const int32_t* __restrict__ key, const float* __restrict__ val, int64_t len,
                                     int32_t* __restrict__ okey, float* __restrict__ oval, int* __restrict__ err) {
  const int lane = lane_id();
  uint64_t v[EPL];
#pragma unroll
  for (int t = 0; t < EPL; ++t) {
    const int e = t * 64 + lane;
    v[t] = e < len ? ((uint64_t(uint32_t(key[e])) << 32) | __float_as_uint(val[e])) : KEY_MAX;
  }
  wave_sort<EPL>(v);
  bool rep = false;
  uint32_t prev_last = 0;
#pragma unroll
  for (int t = 0; t < EPL; ++t) {
    const int e = t * 64 + lane;
    const uint32_t hi = uint32_t(v[t] >> 32);
    // source of element e - 1 (same register): DPP wave_shr:1, lane l <- l - 1
    uint32_t before = uint32_t(__builtin_amdgcn_update_dpp(0, int(hi), 0x138, 0xf, 0xf, false));
    if (lane == 0) before = prev_last;   // ... or the last lane of the previous register
    if (e > 0 && e < len && before == hi) rep = true;
    prev_last = __builtin_amdgcn_readlane(hi, 63);
    if (e < len) {
      okey[e] = int32_t(hi);
      oval[e] = __uint_as_float(uint32_t(v[t]));
    }
  }
  if (rep) atomicOr(err, 1);
}

__global__ __launch_bounds__(256) void sym_sort_out_kernel(const int32_t* __restrict__ nbr,
                                                           const float* __restrict__ Pc, int64_t n, int k,
                                                           int32_t* __restrict__ o_col, float* __restrict__ o_val,
                                                           int* __restrict__ err) {
  const int64_t row = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const int64_t a = row * k;
  wave_bitonic_segment<TSNE_MAX_K / 64>(nbr + a, Pc + a, k, o_col + a, o_val + a, err);
}

// First position in sorted[0..len) whose value is >= x.
__device__ __forceinline__ int64_t lower_bound_i32(const int32_t* __restrict__ sorted, int64_t len, int32_t x) {
  int64_t lo = 0, hi = len;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (sorted[mid] < x) lo = mid + 1;
    else hi = mid;
  }
  return lo;
}

__global__ __launch_bounds__(256) void sym_union_count_kernel(int64_t n, int k, const int32_t* __restrict__ o_col,
                                                              const int64_t* __restrict__ in_ptr,
                                                              const int32_t* __restrict__ s_src,
                                                              int64_t* __restrict__ ucount) {
  const int lane = lane_id();
  const int64_t row = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const int32_t* in = s_src + in_ptr[row];
  const int64_t len = in_ptr[row + 1] - in_ptr[row];
  int dups = 0;
  for (int a0 = 0; a0 < k; a0 += 64) {
    const int a = a0 + lane;
    bool dup = false;
    if (a < k) {
      const int32_t c = o_col[row * k + a];
      const int64_t lb = lower_bound_i32(in, len, c);
      dup = lb < len && in[lb] == c;
    }
    dups += __popcll(__ballot(dup));
  }
  if (lane == 0) ucount[row] = int64_t(k) + len - dups;
}

// Combined value of an entry from its out-weight u and in-weight v (0 when
// absent): MODE 0 the t-SNE average (u + v) / 2n, MODE 1 the fuzzy union.
template <int MODE>
__device__ __forceinline__ float sym_combine(float u, float v, float two_n) {
  if (MODE == 0) return (u + v) / two_n;
  return (u + v) - u * v;
}

template <int MODE>
__global__ __launch_bounds__(256) void sym_write_kernel(int64_t n, int k, const int32_t* __restrict__ o_col,
                                                        const float* __restrict__ o_val,
                                                        const int64_t* __restrict__ in_ptr,
                                                        const int32_t* __restrict__ s_src,
                                                        const float* __restrict__ s_val,
                                                        const int64_t* __restrict__ row_ptr, int32_t* __restrict__ col,
                                                        float* __restrict__ val) {
  const int lane = lane_id();
  const int64_t row = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const float two_n = 2.0f * float(n);
  const int32_t* in = s_src + in_ptr[row];
  const float* inv = s_val + in_ptr[row];
  const int64_t len = in_ptr[row + 1] - in_ptr[row];
  const int32_t* out = o_col + row * k;
  const float* outv = o_val + row * k;
  const int64_t rp = row_ptr[row];
  const uint64_t lt_mask = (uint64_t(1) << lane) - 1;
  // out-entries
  int run = 0;
  for (int a0 = 0; a0 < k; a0 += 64) {
    const int a = a0 + lane;
    bool dup = false;
    int64_t lb = 0;
    int32_t c = 0;
    if (a < k) {
      c = out[a];
      lb = lower_bound_i32(in, len, c);
      dup = lb < len && in[lb] == c;
    }
    const uint64_t m = __ballot(dup);
    if (a < k) {
      const int64_t pos = a + lb - (run + __popcll(m & lt_mask));
      col[rp + pos] = c;
      val[rp + pos] = sym_combine<MODE>(outv[a], dup ? inv[lb] : 0.0f, two_n);
    }
    run += __popcll(m);
  }
  // in-entries not shared with the out-list
  run = 0;
  for (int64_t b0 = 0; b0 < len; b0 += 64) {
    const int64_t b = b0 + lane;
    bool dup = false;
    int64_t lb = 0;
    int32_t c = 0;
    if (b < len) {
      c = in[b];
      lb = lower_bound_i32(out, k, c);
      dup = lb < k && out[lb] == c;
    }
    const uint64_t m = __ballot(dup);
    if (b < len && !dup) {
      const int64_t pos = b + lb - (run + __popcll(m & lt_mask));
      col[rp + pos] = c;
      val[rp + pos] = sym_combine<MODE>(0.0f, inv[b], two_n);
    }
    run += __popcll(m);
  }
}

__global__ __launch_bounds__(256) void sym_tpos_kernel(int64_t n, const int64_t* __restrict__ row_ptr,
                                                       const int32_t* __restrict__ col, int32_t* __restrict__ tpos) {
  const int lane = lane_id();
  const int64_t row = int64_t(blockIdx.x) * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  for (int64_t e = row_ptr[row] + lane; e < row_ptr[row + 1]; e += 64) {
    const int32_t j = col[e];
    int32_t t = -1;
    if (j >= 0 && j < n) {
      const int64_t a = row_ptr[j];
      const int64_t lb = lower_bound_i32(col + a, row_ptr[j + 1] - a, int32_t(row));
      t = int32_t(a + lb);
    }
    tpos[e] = t;
  }
}

__global__ void sym_nnz_kernel(const int64_t* __restrict__ row_ptr, int64_t n, const int* __restrict__ err,
                               int64_t* __restrict__ nnz) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *nnz = *err ? int64_t(-1) : row_ptr[n];
}

struct SymLayout {
  size_t o_err, o_inptr, o_key, o_ent, o_ssrc, o_sval, o_ocol, o_oval, o_ucount, o_bsum, o_rcnt, o_roff, o_rbsum,
      bytes;
  RadixScratch R;
  static SymLayout make(int64_t n, int k) {
    SymLayout L;
    const size_t nk = size_t(n) * size_t(k);
    const size_t nb = size_t(ceil_div(n + 1, SCAN_CHUNK)) + 1;
    Carve c;
    L.o_err = c.take(sizeof(int));
    L.o_inptr = c.take(sizeof(int64_t) * (size_t(n) + 1));
    L.o_key = c.take(sizeof(int32_t) * nk);
    L.o_ent = c.take(sizeof(int32_t) * nk);
    L.o_ssrc = c.take(sizeof(int32_t) * nk);
    L.o_sval = c.take(sizeof(float) * nk);
    // the second buffers of the sort are the out-list buffers, free until
    // the transposed lists are built
    L.o_ocol = c.take(sizeof(int32_t) * nk);
    L.o_oval = c.take(sizeof(float) * nk);
    L.o_ucount = c.take(sizeof(int64_t) * size_t(n));
    L.o_bsum = c.take(sizeof(int64_t) * nb);
    L.R = RadixScratch::make(int64_t(nk));
    L.o_rcnt = c.take(L.R.cnt_bytes);
    L.o_roff = c.take(L.R.off_bytes);
    L.o_rbsum = c.take(L.R.bsum_bytes);
    L.bytes = c.off;
    return L;
  }
  // bits of a target key (0 .. n, n being the invalid bucket)
  static int key_bits(int64_t n) {
    int b = 1;
    while ((int64_t(1) << b) <= n) ++b;
    return b;
  }
};

}  // namespace tsne

namespace tsne {

// The union of the kNN patterns as CSR with the MODE combination of the two
// directed values (steps 1-7 above).
template <int MODE>
int symmetrize_impl(const int32_t* nbr_idx, const float* P_cond, int64_t n, int32_t k, int64_t* row_ptr,
                    int32_t* col, float* val, int32_t* tpos, int64_t* nnz, void* workspace, size_t* workspace_bytes,
                    void* stream) {
  if (!nbr_idx || !P_cond || !row_ptr || !col || !val || !nnz || n < 2 || k < 1 || k >= n) return TSNE_ERR_INVALID_ARG;
  if (k > TSNE_MAX_K) return TSNE_ERR_UNSUPPORTED;
  if (n > (int64_t(1) << 30)) return TSNE_ERR_UNSUPPORTED;  // 2 n k must fit int32 positions in tpos
  if (2 * n * int64_t(k) > (int64_t(1) << 31) - 1) return TSNE_ERR_UNSUPPORTED;
  const SymLayout L = SymLayout::make(n, k);
  int rc = workspace_protocol(workspace, workspace_bytes, L.bytes);
  if (rc >= 0) return rc;
  TSNE_REQUIRE_GFX950();
  char* ws = static_cast<char*>(workspace);
  int* err = reinterpret_cast<int*>(ws + L.o_err);
  int64_t* in_ptr = reinterpret_cast<int64_t*>(ws + L.o_inptr);
  int32_t* key = reinterpret_cast<int32_t*>(ws + L.o_key);
  int32_t* ent = reinterpret_cast<int32_t*>(ws + L.o_ent);
  int32_t* s_src = reinterpret_cast<int32_t*>(ws + L.o_ssrc);
  float* s_val = reinterpret_cast<float*>(ws + L.o_sval);
  int32_t* o_col = reinterpret_cast<int32_t*>(ws + L.o_ocol);
  float* o_val = reinterpret_cast<float*>(ws + L.o_oval);
  int64_t* ucount = reinterpret_cast<int64_t*>(ws + L.o_ucount);
  int64_t* bsum = reinterpret_cast<int64_t*>(ws + L.o_bsum);
  hipStream_t s = as_stream(stream);
  const int64_t nk = n * k;
  const dim3 g_edges(unsigned(ceil_div(nk, 256))), g_rows(unsigned(ceil_div(n, 4))), b(256);

  if ((rc = launch_fill<int>(err, 1, 0, s))) return rc;
  hipLaunchKernelGGL(sym_keys_kernel, g_edges, b, 0, s, nbr_idx, n, k, key, ent, err);
  TSNE_CHECK_LAUNCH();
  bool in_b = false;
  rc = radix_sort_pairs(reinterpret_cast<uint32_t*>(key), ent, reinterpret_cast<uint32_t*>(o_col),
                        reinterpret_cast<int32_t*>(o_val), nk, SymLayout::key_bits(n), L.R,
                        reinterpret_cast<uint32_t*>(ws + L.o_rcnt), reinterpret_cast<int64_t*>(ws + L.o_roff),
                        reinterpret_cast<int64_t*>(ws + L.o_rbsum), s, in_b);
  if (rc) return rc;
  // the sorted targets and entries (in the out-list buffers after an odd
  // number of passes)
  const int32_t* skey = in_b ? o_col : key;
  const int32_t* sent = in_b ? reinterpret_cast<const int32_t*>(o_val) : ent;
  hipLaunchKernelGGL(sym_inptr_kernel, dim3(unsigned(ceil_div(nk + 1, 256))), b, 0, s, skey, nk, n, in_ptr);
  TSNE_CHECK_LAUNCH();
  hipLaunchKernelGGL(sym_lists_kernel, g_edges, b, 0, s, skey, sent, P_cond, in_ptr, n, k, s_src, s_val, err);
  TSNE_CHECK_LAUNCH();
  hipLaunchKernelGGL(sym_sort_out_kernel, g_rows, b, 0, s, nbr_idx, P_cond, n, k, o_col, o_val, err);
  TSNE_CHECK_LAUNCH();
  hipLaunchKernelGGL(sym_union_count_kernel, g_rows, b, 0, s, n, k, o_col, in_ptr, s_src, ucount);
  TSNE_CHECK_LAUNCH();
  if ((rc = exclusive_scan<int64_t>(ucount, n, row_ptr, bsum, s))) return rc;
  hipLaunchKernelGGL(sym_write_kernel<MODE>, g_rows, b, 0, s, n, k, o_col, o_val, in_ptr, s_src, s_val, row_ptr, col,
                     val);
  TSNE_CHECK_LAUNCH();
  if (tpos) {
    hipLaunchKernelGGL(sym_tpos_kernel, g_rows, b, 0, s, n, row_ptr, col, tpos);
    TSNE_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(sym_nnz_kernel, dim3(1), dim3(64), 0, s, row_ptr, n, err, nnz);
  TSNE_CHECK_LAUNCH();
  return TSNE_OK;
}

}  // namespace tsne

extern "C" int tsne_symmetrize(const int32_t* nbr_idx, const float* P_cond, int64_t n, int32_t k, int64_t* row_ptr,
                               int32_t* col, float* val, int32_t* tpos, int64_t* nnz, void* workspace,
                               size_t* workspace_bytes, void* stream) {
  return tsne::symmetrize_impl<0>(nbr_idx, P_cond, n, k, row_ptr, col, val, tpos, nnz, workspace, workspace_bytes,
                                  stream);
}

extern "C" int tsne_umap_fuzzy_union(const int32_t* nbr_idx, const float* w, int64_t n, int32_t k, int64_t* row_ptr,
                                     int32_t* col, float* val, int32_t* tpos, int64_t* nnz, void* workspace,
                                     size_t* workspace_bytes, void* stream) {
  return tsne::symmetrize_impl<1>(nbr_idx, w, n, k, row_ptr, col, val, tpos, nnz, workspace, workspace_bytes, stream);
}
