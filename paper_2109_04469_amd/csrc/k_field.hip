// Field kernel: the field step of arXiv:2109.04469, Sec. 2 steps 1-2, in one
// workgroup (field_block.h).
#include "field_block.h"
#include "pic_internal.h"

namespace pic {

__global__ __launch_bounds__(kFieldThreads) void k_field(FieldArgs a) { field_block(a); }

hipError_t launch_field(const FieldArgs& a, hipStream_t s) {
  if (a.nx > kMaxNx || a.nx < 3) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_field, dim3(1), dim3(kFieldThreads), 0, s, a);
  return hipGetLastError();
}

// Workgroups 1.. of k_field_cand (2.. when workgroup 1 writes the records),
// the wg-th of nwg: bit i of word i / 32 is the collision candidacy of
// electron slot i of the step f.cand_step (Philox word i mod 4 of the block
// (step, i / 4, 4, 0) below the threshold), for the slots the deciding pass
// outputs: the sum of its tile totals' output counts.
__device__ void candidacy_bits(const FieldArgs& f, int wg, int nwg) {
  __shared__ unsigned long long s_w[kFieldThreads / kWave];
  const int tid = threadIdx.x;
  // tiles of the deciding pass (its slot count), four loads per thread in
  // flight at a time
  int64_t np = *f.cand_count;
  if (np > f.cand_cap) np = f.cand_cap;
  const int64_t ntiles = (np + kTile - 1) / kTile;
  unsigned long long own = 0;
  for (int64_t t0 = tid; t0 < ntiles; t0 += 4 * kFieldThreads) {
    uint64_t v[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const int64_t t = t0 + (int64_t)k * kFieldThreads;
      v[k] = t < ntiles ? f.cand_tcnt[t] : 0ull;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) own += v[k] & 0xFFFFull;
  }
  own = wave_sum<unsigned long long>(own);
  if ((tid & (kWave - 1)) == 0) s_w[tid / kWave] = own;
  __syncthreads();
  int64_t n = 0;
  for (int w = 0; w < kFieldThreads / kWave; ++w) n += (int64_t)s_w[w];
  if (n > f.cand_cap) n = f.cand_cap;
  const int64_t words = (n + 31) / 32;
  for (int64_t wi = (int64_t)wg * kFieldThreads + tid; wi < words;
       wi += (int64_t)nwg * kFieldThreads) {
    uint32_t bits = 0;
#pragma unroll
    for (int g = 0; g < 8; ++g) {
      const uint4 r = draw(f.cand_step, (uint32_t)(wi * 8 + g), 0, 4, f.seed, f.run);
      bits |= ((uint64_t)r.x < f.cand_thr ? 1u : 0u) << (4 * g);
      bits |= ((uint64_t)r.y < f.cand_thr ? 1u : 0u) << (4 * g + 1);
      bits |= ((uint64_t)r.z < f.cand_thr ? 1u : 0u) << (4 * g + 2);
      bits |= ((uint64_t)r.w < f.cand_thr ? 1u : 0u) << (4 * g + 3);
    }
    f.cand[wi] = bits;
  }
}

// Workgroup 1 of k_field_cand: where each workgroup of the fused electron
// pass that follows starts. That kernel gives workgroup b of its grid g a
// contiguous run of tiles, one tile more for b < ntiles mod g; its record
// holds the run, the outputs, births and queued slots of all tiles before
// it (from the deciding pass's tile totals) and the pass's slot and ion
// counts. Each thread sums a contiguous run of tile totals, a block scan
// gives the prefix at its start, and the thread walks its run writing the
// record of every workgroup whose first tile lies there.
__device__ void emit_records(const FieldArgs& f) {
  __shared__ i128p s_w128[kFieldWaves + 1];
  constexpr int kRun = 8;  // tile totals per thread kept in registers
  const int tid = threadIdx.x;
  // the thread's run length comes from the tile capacity, so that its first
  // totals are requested together with the counts
  const int per = (int)((f.cand_zero_n + kFieldThreads - 1) / kFieldThreads);
  const int u0 = tid * per;
  int64_t n = *f.cand_count;
  const int64_t nion = *f.rec_nion;
  uint64_t v[kRun];
#pragma unroll
  for (int k = 0; k < kRun; ++k)
    v[k] = k < per && u0 + k < f.cand_zero_n ? f.cand_tcnt[u0 + k] : 0ull;
  if (n > f.cand_cap) n = f.cand_cap;
  const int ntiles = (int)((n + kTile - 1) / kTile);
  const int g = f.rec_grid;
  const int q = ntiles / g, r = ntiles % g;
  const int u1 = min(u0 + per, ntiles);
  // outputs, and births << 32 | queued slots (each total below 2^31), as
  // the high and low words of one 128-bit scan (no carry between them)
  int64_t so = 0, sbr = 0;
#pragma unroll
  for (int k = 0; k < kRun; ++k)
    if (u0 + k < u1) {
      so += (int64_t)(v[k] & 0xFFFFull);
      sbr += (int64_t)((((v[k] >> 16) & 0xFFFFull) << 32) | (v[k] >> 32));
    }
  for (int u = u0 + kRun; u < u1; ++u) {
    const uint64_t w = f.cand_tcnt[u];
    so += (int64_t)(w & 0xFFFFull);
    sbr += (int64_t)((((w >> 16) & 0xFFFFull) << 32) | (w >> 32));
  }
  i128p tot, ex;
  tot.lo = (uint64_t)sbr;
  tot.hi = so;
  block_excl_scan128(tot, ex, s_w128);
  int64_t eo = ex.hi, ebr = (int64_t)ex.lo;
  // the first workgroup whose run starts at or after u0, and its first tile
  // (then stepped along without divisions)
  int b = 0, bt = 0;
  if (u0 < u1) {
    const int split = r * (q + 1);
    if (u0 <= split) {
      b = (u0 + q) / (q + 1);
      bt = b * (q + 1);
    } else {
      b = r + (u0 - split + q - 1) / q;
      bt = split + (b - r) * q;
    }
  }
  // the record of every workgroup whose first tile is u
  auto visit = [&](int u, uint64_t w) {
    if (u == bt) {
      WgRec rec{};
      rec.pref_o = eo;
      rec.pref_b = (int64_t)((uint64_t)ebr >> 32);
      rec.pref_r = (int64_t)((uint64_t)ebr & 0xFFFFFFFFull);
      rec.n_tot = n;
      rec.bbase = nion;
      rec.t0 = u;
      rec.t1 = u + (b < r ? q + 1 : q);
      f.rec[b] = rec;
      bt = rec.t1;
      ++b;
    }
    eo += (int64_t)(w & 0xFFFFull);
    ebr += (int64_t)((((w >> 16) & 0xFFFFull) << 32) | (w >> 32));
  };
#pragma unroll
  for (int k = 0; k < kRun; ++k)
    if (u0 + k < u1) visit(u0 + k, v[k]);
  for (int u = u0 + kRun; u < u1; ++u) visit(u, f.cand_tcnt[u]);
  // workgroups without tiles (fewer tiles than workgroups)
  if (q == 0) {
    for (int e = r + tid; e < g; e += kFieldThreads) {
      WgRec rec{};
      rec.n_tot = n;
      rec.bbase = nion;
      rec.t0 = rec.t1 = ntiles;
      f.rec[e] = rec;
    }
  }
}

// Also, for the fused electron pass that follows: its tile totals buffer
// zeroed, its workgroup records (emit_records) and the first pool entries
// of its births (the pools' fill levels before it), which its workgroups
// read while its last tile advances them. Launched with 1 + num_cu
// workgroups (at least 3).
__global__ __launch_bounds__(kFieldThreads) void k_field_cand(FieldArgs a) {
  if (blockIdx.x == 0) {
    if (threadIdx.x == 0) {
      a.ctl->pbase[0] = a.ctl->pool_n[0];
      a.ctl->pbase[1] = a.ctl->pool_n[1];
    }
    field_block(a);
  } else {
    // workgroup 1 writes the records alone (with the candidacy bits as
    // well it would finish after the field); the rest draw the bits
    if (blockIdx.x == 1 && a.rec) {
      emit_records(a);
      return;
    }
    const int w0 = a.rec ? 2 : 1;
    for (int64_t i = (int64_t)(blockIdx.x - w0) * kFieldThreads + threadIdx.x; i < a.cand_zero_n;
         i += (int64_t)(gridDim.x - w0) * kFieldThreads)
      a.cand_zero[i] = 0ull;
    candidacy_bits(a, (int)blockIdx.x - w0, (int)gridDim.x - w0);
  }
}

hipError_t launch_field_cand(const FieldArgs& a, int num_cu, hipStream_t s) {
  if (a.nx > kMaxNx || a.nx < 3 || !a.cand || !a.cand_tcnt || !a.cand_zero || num_cu < 1 ||
      (a.rec && (a.rec_grid < 1 || a.rec_grid > a.cand_zero_n || !a.rec_nion)))
    return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_field_cand, dim3(1 + (num_cu < 2 ? 2 : num_cu)), dim3(kFieldThreads), 0, s, a);
  return hipGetLastError();
}

// the fields of n discharges, one workgroup each
__global__ __launch_bounds__(kFieldThreads) void k_field_b(const FieldArgs* __restrict__ f) {
  field_block(f[blockIdx.x]);
}

hipError_t launch_batch_field(const FieldArgs* f, int n, hipStream_t s) {
  if (n < 1 || n > kMaxBatch) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_field_b, dim3(n), dim3(kFieldThreads), 0, s, f);
  return hipGetLastError();
}

}  // namespace pic
