// Setup kernels of the bootstrap AMG hierarchy:
//  * B = I - A assembly and input validation (Section 2),
//  * C/F splitting: geometric (Section 7) or a greedy maximal independent set
//    computed in parallel rounds (stand-in for compatible relaxation),
//  * interpolation sets J_i and the patterns of P (eq. Pstructure), Q^T,
//  * Galerkin products Q B P, Q M Q^T, P^T N P (Algorithm 1): an integer
//    symbolic phase (sorted patterns, bit-exact) and a numeric phase,
//  * the batched small weighted least-squares fits of eq. ls_interpolation
//    with the sum-to-one constraint of Section 5,
//  * relaxation of the r test-vector pairs and the reductions for sigma
//    (eq. singular_value), the normalisation and the LS weights
//    (eq. ls_weights).
#include <algorithm>

#include "bamg_internal.h"
#include "device_common.h"

namespace bamg {

// ============================================================ assembly
__global__ void k_b_count(const int *__restrict__ rp, const int *__restrict__ ci, int n,
                          int *__restrict__ cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int has = 0;
  for (int k = rp[i]; k < rp[i + 1]; ++k) has |= (ci[k] == i);
  cnt[i] = rp[i + 1] - rp[i] + (has ? 0 : 1);
}

// B = I - A, diagonal inserted in column order when A has none
__global__ void k_b_fill(const int *__restrict__ rp, const int *__restrict__ ci,
                         const double *__restrict__ a, int n, const int *__restrict__ brp,
                         int *__restrict__ bci, double *__restrict__ bv) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int p = brp[i];
  bool placed = false;
  for (int k = rp[i]; k < rp[i + 1]; ++k) {
    const int j = ci[k];
    if (!placed && j > i) {
      bci[p] = i;
      bv[p++] = 1.0;
      placed = true;
    }
    bci[p] = j;
    bv[p++] = (j == i ? 1.0 : 0.0) - a[k];
    if (j == i) placed = true;
  }
  if (!placed) {
    bci[p] = i;
    bv[p] = 1.0;
  }
}

// Checks of the input CSR: indices in range and strictly ascending (flag
// bit 0), entries non-negative (bit 1), entries finite (bit 2).
__global__ void k_check_csr(const int *__restrict__ rp, const int *__restrict__ ci,
                            const double *__restrict__ a, int n, int nnz, int *__restrict__ flag) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int b = rp[i], e = rp[i + 1];
  if (b < 0 || e < b || e > nnz) {
    atomicOr(flag, 1);
    return;
  }
  for (int k = b; k < e; ++k) {
    const int j = ci[k];
    if (j < 0 || j >= n || (k > b && j <= ci[k - 1])) atomicOr(flag, 1);
    const double v = a[k];
    if (!isfinite(v)) atomicOr(flag, 4);
    else if (!(v >= 0.0)) atomicOr(flag, 2);
  }
}

void build_B(const int *arp, const int *aci, const double *aval, int n, Pool &pool, Csr &B,
             double *&bval, hipStream_t s) {
  int *cnt = pool.get<int>(n);
  k_b_count<<<ceil_div(n, 256), 256, 0, s>>>(arp, aci, n, cnt);
  LAUNCHCHK();
  B.nr = B.nc = n;
  B.rp = pool.get<int>(n + 1);
  scan_counts(pool, cnt, B.rp, n, s);
  B.nnz = read_int(B.rp + n, s);
  B.ci = pool.get<int>(B.nnz);
  bval = pool.get<double>(B.nnz);
  k_b_fill<<<ceil_div(n, 256), 256, 0, s>>>(arp, aci, aval, n, B.rp, B.ci, bval);
  LAUNCHCHK();
  pool.release(cnt);
}

// Column sums of A through the rows of B^T: sum_i a_ij = sum_i (delta_ij - B_ij).
__global__ void k_colsum_check(const int *__restrict__ trp, const int *__restrict__ tci,
                               const double *__restrict__ tv, int n, int *__restrict__ flag) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  double s = 0.0;
  for (int k = trp[j]; k < trp[j + 1]; ++k) s += (tci[k] == j ? 1.0 : 0.0) - tv[k];
  if (!(fabs(s - 1.0) <= 1e-12)) atomicOr(flag, 2);
}

// Reachability from state 0, forward (rows of B) and backward (rows of B^T),
// in two forms.
//
// LDS form (n up to about 1.3 M states): one workgroup per direction,
// level-synchronous breadth-first search with the visited bitmap in LDS and
// the frontier queues in global memory.
//
// Global form (larger chains): the visited bitmap in global memory (n / 8
// bytes per direction) and one launch per frontier level, each with many
// workgroups per direction, so the scattered claims and row loads of a level
// are spread over many CUs instead of the memory pipeline of one; the kernel
// boundaries order the levels (no grid barrier, no co-residency needed). The
// order of the search does not matter for the visited set, so each thread
// follows the states it claims depth first, up to kReachDepth hops and
// kReachStack pending states (a per-thread stack in LDS), and hands the rest
// to the next level's frontier: far fewer levels than the graph's diameter.
// A neighbour's row pointers are loaded together with the atomic that claims
// it (used only if the claim succeeds), so a hop is two dependent round
// trips, not three. Every state is claimed once, so every stack and every
// frontier is finite, and at most n + 1 levels are non-empty. The states
// reached are counted from the bitmap at the end.
constexpr int kReachDepth = 32, kReachStack = 10, kReachStateBits = 26;
constexpr int kReachThreads = 256, kReachBlocks = 64;  // global form, per direction
// Levels enqueued with the setup: kReachFirst when the search starts, the
// rest up to kReachLevels by reach_more once the setup's own stream holds a
// long queue of work (so the host time of those launches does not delay the
// setup), more at the join if the search needs them.
constexpr int kReachFirst = 32, kReachLevels = 512;

__global__ void __launch_bounds__(1024)
    k_reach_lds(const int *__restrict__ rp0, const int *__restrict__ ci0,
                const int *__restrict__ rp1, const int *__restrict__ ci1, int n,
                int *__restrict__ queues, int *__restrict__ out) {
  extern __shared__ unsigned lbits[];
  __shared__ int cur_n, nxt_n, found;
  const int b = blockIdx.x, t = threadIdx.x;
  const int *rp = b ? rp1 : rp0, *ci = b ? ci1 : ci0;
  const int words = (n + 31) >> 5;
  int *qa = queues + (size_t)b * 2 * n, *qb = qa + n;
  for (int i = t; i < words; i += blockDim.x) lbits[i] = i == 0 ? 1u : 0u;
  if (t == 0) {
    qa[0] = 0;
    cur_n = 1;
    nxt_n = 0;
    found = 0;
  }
  __syncthreads();
  int *cur = qa, *nxt = qb;
  while (cur_n > 0) {
    const int cn = cur_n;
    int mine = 0;
    for (int idx = t; idx < cn; idx += blockDim.x) {
      const int v0 = cur[idx];
      const int kb = rp[v0], ke = rp[v0 + 1];
      for (int k = kb; k < ke; k += 4) {
        int us[4];
        unsigned old[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) us[j] = ci[min(k + j, ke - 1)];
#pragma unroll
        for (int j = 0; j < 4; ++j)
          old[j] = k + j < ke ? atomicOr(&lbits[us[j] >> 5], 1u << (us[j] & 31)) : ~0u;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          if (k + j >= ke || (old[j] >> (us[j] & 31)) & 1u) continue;
          ++mine;
          nxt[atomicAdd(&nxt_n, 1)] = us[j];
        }
      }
    }
    if (mine) atomicAdd(&found, mine);
    __syncthreads();
    if (t == 0) {
      cur_n = nxt_n;
      nxt_n = 0;
    }
    __syncthreads();
    int *tmp = cur;
    cur = nxt;
    nxt = tmp;
  }
  if (t == 0) out[b] = 1 + found;
}

// Global form. ctl + 32 d (a cache line of its own) holds the frontier
// sizes of direction d for the levels k = 0, 1, 2 (mod 3); direction d's
// queues are queues + 2 d n (level k reads half k & 1 and appends to the
// other).
__global__ void k_reach_init(unsigned *__restrict__ visited, int *__restrict__ queues,
                             int *__restrict__ ctl, int n) {
  const long words = (n + 31) >> 5;
  const long t = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < 2 * words) visited[t] = t % words == 0 ? 1u : 0u;
  if (t < 2) {
    queues[(size_t)t * 2 * n] = 0;
    ctl[32 * t] = 1;
    ctl[32 * t + 1] = 0;
    ctl[32 * t + 2] = 0;
  }
}

// Level `level` of both directions: blocks [0, kReachBlocks) forward, the
// rest backward. Returns at once when the level's frontier is empty.
__global__ void __launch_bounds__(kReachThreads)
    k_reach_level(const int *__restrict__ rp0, const int *__restrict__ ci0,
                  const int *__restrict__ rp1, const int *__restrict__ ci1, int n,
                  unsigned *__restrict__ visited, int *__restrict__ queues,
                  int *__restrict__ ctl, int level) {
  __shared__ int stk_all[kReachThreads * 3 * kReachStack];
  const int d = blockIdx.x / kReachBlocks, wg = blockIdx.x % kReachBlocks;
  int *c = ctl + 32 * d;
  const int cn = c[level % 3];
  // the counter the next level appends to holds the previous level's
  // frontier size, which no block of this launch reads; it is cleared by
  // every level, empty ones included, so a direction that has finished
  // keeps reading empty frontiers while the other goes on
  if (wg == 0 && threadIdx.x == 0) c[(level + 2) % 3] = 0;
  if (cn == 0) return;
  const int *rp = d ? rp1 : rp0, *ci = d ? ci1 : ci0;
  const size_t words = (size_t)((n + 31) >> 5);
  unsigned *bits = visited + d * words;
  const int *cur = queues + (size_t)d * 2 * n + (size_t)(level & 1) * n;
  int *nxt = queues + (size_t)d * 2 * n + (size_t)((level + 1) & 1) * n;
  int *nxt_n = c + (level + 1) % 3;
  int *stk = stk_all + threadIdx.x * 3 * kReachStack;
  for (int idx = wg * kReachThreads + threadIdx.x; idx < cn; idx += kReachBlocks * kReachThreads) {
    int sp = 0, dep = 0;
    const int v0 = cur[idx];
    int kb = rp[v0], ke = rp[v0 + 1];
    for (;;) {
      // four neighbours per round: their indices are loaded together
      // (positions past the row end reload its last entry and are skipped)
      for (int k = kb; k < ke; k += 4) {
        int us[4], r0[4], r1[4];
        unsigned old[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) us[j] = ci[min(k + j, ke - 1)];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int u = us[j];
          old[j] = k + j < ke ? atomicOr(&bits[u >> 5], 1u << (u & 31)) : ~0u;
          r0[j] = rp[u];
          r1[j] = rp[u + 1];
        }
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int u = us[j];
          if (k + j >= ke || (old[j] >> (u & 31)) & 1u) continue;
          if (dep + 1 < kReachDepth && sp < kReachStack) {
            stk[3 * sp] = dep + 1;
            stk[3 * sp + 1] = r0[j];
            stk[3 * sp + 2] = r1[j];
            ++sp;
          } else {
            // one atomic per wave for the lanes appending here together
            const unsigned long long act = __ballot(1);
            const int leader = __ffsll((long long)act) - 1;
            int base = 0;
            if (threadIdx.x % kWave == leader) base = atomicAdd(nxt_n, __popcll(act));
            base = __shfl(base, leader);
            nxt[base + __popcll(act & ((1ull << (threadIdx.x % kWave)) - 1))] = u;
          }
        }
      }
      if (sp == 0) break;
      --sp;
      dep = stk[3 * sp];
      kb = stk[3 * sp + 1];
      ke = stk[3 * sp + 2];
    }
  }
}

// out[d] += states set in direction d's bitmap; grid (blocks, 2)
__global__ void k_reach_count(const unsigned *__restrict__ visited, int n, int *__restrict__ out) {
  __shared__ int sh[4];
  const long words = (n + 31) >> 5;
  const unsigned *bits = visited + blockIdx.y * words;
  int cnt = 0;
  for (long w = (long)blockIdx.x * blockDim.x + threadIdx.x; w < words;
       w += (long)gridDim.x * blockDim.x)
    cnt += __popc(bits[w]);
  for (int o = kWave / 2; o > 0; o >>= 1) cnt += __shfl_xor(cnt, o);
  if (threadIdx.x % kWave == 0) sh[threadIdx.x / kWave] = cnt;
  __syncthreads();
  if (threadIdx.x == 0) atomicAdd(&out[blockIdx.y], sh[0] + sh[1] + sh[2] + sh[3]);
}

static void reach_levels(const Csr &B, const Csr &Bt, unsigned *visited, int *queues, int k0,
                         int k1, hipStream_t s) {
  const int n = B.nr;
  int *ctl = queues + 4 * (size_t)n;
  for (int k = k0; k < k1; ++k) {
    k_reach_level<<<2 * kReachBlocks, kReachThreads, 0, s>>>(B.rp, B.ci, Bt.rp, Bt.ci, n,
                                                             visited, queues, ctl, k);
    LAUNCHCHK();
  }
}

static void reach_count(unsigned *visited, int n, int *flag, hipStream_t s) {
  k_reach_count<<<dim3(64, 2), 256, 0, s>>>(visited, n, flag + 1);
  LAUNCHCHK();
}

// Launch the reachability search on stream s (the caller's auxiliary
// stream); the states reached each way are added to flag[1], flag[2] (zero
// before). queues: 4 n + 64 ints. Returns the number of levels enqueued in the
// global form (finish with reach_finish), 0 for the LDS form.
int reach_launch(const Csr &B, const Csr &Bt, unsigned *visited, int *queues, int *flag,
                 bool force_global, hipStream_t s) {
  const int n = B.nr;
  const size_t shm = sizeof(unsigned) * (size_t)((n + 31) / 32);
  int dev = 0, maxlds = 65536;
  HIPCHK(hipGetDevice(&dev));
  HIPCHK(hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
  if (n >= (1 << kReachStateBits)) fail(BAMG_E_ARG, "reachability search: more than 2^26 states");
  if (!force_global && shm + 256 <= (size_t)maxlds) {
    HIPCHK(hipFuncSetAttribute((const void *)k_reach_lds,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));
    k_reach_lds<<<2, 1024, shm, s>>>(B.rp, B.ci, Bt.rp, Bt.ci, n, queues, flag + 1);
    LAUNCHCHK();
    return 0;
  }
  const long words = (n + 31) / 32;
  k_reach_init<<<ceil_div(2 * words, 256), 256, 0, s>>>(visited, queues, queues + 4 * (size_t)n,
                                                        n);
  LAUNCHCHK();
  reach_levels(B, Bt, visited, queues, 0, kReachFirst, s);
  reach_count(visited, n, flag, s);
  return kReachFirst;
}

// Levels k0 .. kReachLevels - 1 of a global-form search started by
// reach_launch on the same stream s, then the reached states counted again.
// Returns the number of levels now enqueued.
int reach_more(const Csr &B, const Csr &Bt, unsigned *visited, int *queues, int *flag, int k0,
               hipStream_t s) {
  if (k0 >= kReachLevels) return k0;
  reach_levels(B, Bt, visited, queues, k0, kReachLevels, s);
  fill_i32(flag + 1, 0, 2, s);
  reach_count(visited, B.nr, flag, s);
  return kReachLevels;
}

// After the work reach_launch enqueued has completed: a graph whose search
// needs more than the enqueued levels (a long path: about one level per
// kReachDepth states) gets further levels, 256 per host check, and is
// counted again. Runs on stream s; returns when the counts in flag are final.
void reach_finish(const Csr &B, const Csr &Bt, unsigned *visited, int *queues, int *flag,
                  int levels, hipStream_t s) {
  if (levels <= 0) return;
  const int n = B.nr;
  int *ctl = queues + 4 * (size_t)n;
  bool more = false;
  for (;;) {
    int hc[64];
    HIPCHK(hipMemcpyAsync(hc, ctl, sizeof(hc), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (hc[levels % 3] == 0 && hc[32 + levels % 3] == 0) break;
    reach_levels(B, Bt, visited, queues, levels, levels + 256, s);
    levels += 256;
    more = true;
  }
  if (more) {
    fill_i32(flag + 1, 0, 2, s);
    reach_count(visited, n, flag, s);
  }
}

// Structural checks of the caller's CSR (indices in range, ascending,
// values finite and non-negative) before anything indexes through it.
int check_input(Pool &pool, const int *arp, const int *aci, const double *aval, int n, int nnz,
                hipStream_t s) {
  int *ends = pool.pinned();
  HIPCHK(hipMemcpyAsync(&ends[0], arp, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&ends[1], arp + n, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (ends[0] != 0 || ends[1] != nnz) return BAMG_E_ARG;
  int *flag = pool.get<int>(1);
  fill_i32(flag, 0, 1, s);
  k_check_csr<<<ceil_div(n, 256), 256, 0, s>>>(arp, aci, aval, n, nnz, flag);
  LAUNCHCHK();
  const int f = read_int(flag, s);
  pool.release(flag);
  if (f & 1) return BAMG_E_ARG;
  if (f & 4) return BAMG_E_NONFINITE;
  if (f & 2) return BAMG_E_NOT_STOCHASTIC;
  return BAMG_OK;
}

// Column sums of A equal to 1 (through B^T, whose values btv are B's
// permuted): flag[0] bit 1 on failure. Enqueued on s, read at the join.
void colsum_launch(const Csr &Bt, const double *btv, int *flag, hipStream_t s) {
  k_colsum_check<<<ceil_div(Bt.nr, 256), 256, 0, s>>>(Bt.rp, Bt.ci, btv, Bt.nr, flag);
  LAUNCHCHK();
}

// Status from the validation flags (host copy): stochastic columns, then
// strong connectivity (all states reached from state 0 both ways).
int validation_status(const int *h, int n) {
  if (h[0] & 2) return BAMG_E_NOT_STOCHASTIC;
  if (h[1] != n || h[2] != n) return BAMG_E_REDUCIBLE;
  return BAMG_OK;
}

// ============================================================ graph
// G = pattern(B + B^T) without the diagonal: merge of row i of B and of B^T.
template <bool FILL>
__global__ void k_sym_graph(const int *__restrict__ brp, const int *__restrict__ bci,
                            const int *__restrict__ trp, const int *__restrict__ tci, int n,
                            int *__restrict__ cnt, const int *__restrict__ grp,
                            int *__restrict__ gci) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int a = brp[i], ae = brp[i + 1], b = trp[i], be = trp[i + 1];
  int c = 0, p = FILL ? grp[i] : 0;
  while (a < ae || b < be) {
    int j;
    if (b >= be || (a < ae && bci[a] < tci[b])) {
      j = bci[a++];
    } else if (a >= ae || tci[b] < bci[a]) {
      j = tci[b++];
    } else {
      j = bci[a++];
      ++b;
    }
    if (j == i) continue;
    if (FILL)
      gci[p++] = j;
    else
      ++c;
  }
  if (!FILL) cnt[i] = c;
}

void sym_graph(Pool &pool, const Csr &B, const Csr &Bt, Csr &G, hipStream_t s) {
  const int n = B.nr;
  int *cnt = pool.get<int>(n);
  k_sym_graph<false><<<ceil_div(n, 256), 256, 0, s>>>(B.rp, B.ci, Bt.rp, Bt.ci, n, cnt, nullptr,
                                                      nullptr);
  LAUNCHCHK();
  G.nr = G.nc = n;
  G.rp = pool.get<int>(n + 1);
  scan_counts(pool, cnt, G.rp, n, s);
  G.nnz = read_int(G.rp + n, s);
  G.ci = pool.get<int>(G.nnz);
  k_sym_graph<true><<<ceil_div(n, 256), 256, 0, s>>>(B.rp, B.ci, Bt.rp, Bt.ci, n, nullptr, G.rp,
                                                     G.ci);
  LAUNCHCHK();
  pool.release(cnt);
}

// ============================================================ C/F splitting
// Geometric: on a grid every other point in each direction (Section 7);
// on a line every other point.
__global__ void k_geom_cf(int n, int nx, int gkind, int *__restrict__ cf) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (gkind == 2) {
    const int ix = i % nx, iy = i / nx;
    cf[i] = ((ix & 1) == 0 && (iy & 1) == 0) ? 1 : 0;
  } else {
    cf[i] = (i & 1) == 0 ? 1 : 0;
  }
}

void geom_cf(int n, int nx, int gkind, int *cf, hipStream_t s) {
  k_geom_cf<<<ceil_div(n, 256), 256, 0, s>>>(n, nx, gkind, cf);
  LAUNCHCHK();
}

// Greedy maximal independent set in decreasing priority (key_i, i), key_i
// the first Philox word of counter (i, level, 2, 0), key (seed, 0).
// Computed in rounds: an undecided vertex whose priority exceeds that of
// every undecided neighbour joins; then the neighbours of the new members
// leave. Every round reproduces a prefix of the sequential greedy order, so
// the result is the same set (lexicographically-first MIS).
__global__ void k_mis_keys(int n, uint64_t seed, int level, uint64_t *__restrict__ key,
                           int *__restrict__ state) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  key[i] = philox_word0((uint64_t)i, (uint64_t)level, 2, 0, seed, 0);
  state[i] = -1;
}

__global__ void k_mis_select(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                             const uint64_t *__restrict__ key, const int *__restrict__ state,
                             int *__restrict__ sel, int round) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n || state[v] != -1) return;
  const uint64_t kv = key[v];
  for (int k = rp[v]; k < rp[v + 1]; ++k) {
    const int u = ci[k];
    if (state[u] != -1) continue;
    const uint64_t ku = key[u];
    if (ku > kv || (ku == kv && u > v)) return;
  }
  sel[v] = round;
}

__global__ void k_mis_update(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                             const int *__restrict__ sel, int *__restrict__ state, int round,
                             int *__restrict__ undecided) {
  const int v = blockIdx.x * blockDim.x + threadIdx.x;
  bool und = false;
  if (v < n && state[v] == -1) {
    if (sel[v] == round) {
      state[v] = 1;
    } else {
      bool beaten = false;
      for (int k = rp[v]; k < rp[v + 1] && !beaten; ++k) beaten = sel[ci[k]] == round;
      if (beaten)
        state[v] = 0;
      else
        und = true;
    }
  }
  const unsigned long long b = __ballot(und);  // one counter update per wave
  if ((threadIdx.x % kWave) == 0 && b) atomicAdd(undecided, (int)__popcll(b));
}

// Rounds of k_mis_select / k_mis_update until no vertex with state -1 is
// left: the greedy independent set, in decreasing (key, index) order, of
// the vertices that start undecided (-1); other states are left alone.
void mis_rounds(Pool &pool, const Csr &G, const uint64_t *key, int *state, hipStream_t s) {
  const int n = G.nr;
  int *sel = pool.get<int>(n);
  int *und = pool.get<int>(1);
  fill_i32(sel, 0, n, s);
  // Two rounds per host check of the undecided count: a round after the
  // last decision changes nothing, so the set is the same, with half the
  // host round trips.
  for (int round = 1;; round += 2) {
    if (round > n + 1) fail(BAMG_E_DEVICE, "MIS did not terminate");
    for (int q = 0; q < 2; ++q) {
      fill_i32(und, 0, 1, s);
      k_mis_select<<<ceil_div(n, 256), 256, 0, s>>>(n, G.rp, G.ci, key, state, sel, round + q);
      LAUNCHCHK();
      k_mis_update<<<ceil_div(n, 256), 256, 0, s>>>(n, G.rp, G.ci, sel, state, round + q, und);
      LAUNCHCHK();
    }
    if (read_int(und, s) == 0) break;
  }
  pool.release(sel);
  pool.release(und);
}

void mis_cf(Pool &pool, const Csr &G, uint64_t seed, int level, int *cf, hipStream_t s) {
  const int n = G.nr;
  uint64_t *key = pool.get<uint64_t>(n);
  k_mis_keys<<<ceil_div(n, 256), 256, 0, s>>>(n, seed, level, key, cf);
  LAUNCHCHK();
  mis_rounds(pool, G, key, cf, s);
  pool.release(key);
}

__global__ void k_cidx(const int *__restrict__ cf, const int *__restrict__ scan, int n,
                       int *__restrict__ cidx, int *__restrict__ cpts) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  if (cf[i]) {
    cidx[i] = scan[i];
    cpts[scan[i]] = i;
  } else {
    cidx[i] = -1;
  }
}

int coarse_numbering(Pool &pool, const int *cf, int n, int *cidx, int *&cpts, hipStream_t s) {
  int *sc = pool.get<int>(n + 1);
  scan_counts(pool, cf, sc, n, s);
  const int nc = read_int(sc + n, s);
  cpts = pool.get<int>(nc);
  k_cidx<<<ceil_div(n, 256), 256, 0, s>>>(cf, sc, n, cidx, cpts);
  LAUNCHCHK();
  pool.release(sc);
  return nc;
}

// ============================================================ J_i and P
// Geometric J_i: coarse points within Chebyshev distance 1 (grid) or the
// two neighbours (line), ascending coarse index, at most cap.
// Algebraic J_i: coarse neighbours in G ranked by the number of common
// neighbours (ties: smaller index), at most cap, then sorted by coarse index.
__device__ int common_neighbours(const int *__restrict__ rp, const int *__restrict__ ci, int i,
                                 int j) {
  int a = rp[i], ae = rp[i + 1], b = rp[j], be = rp[j + 1], c = 0;
  while (a < ae && b < be) {
    const int x = ci[a], y = ci[b];
    if (x == y) {
      ++c;
      ++a;
      ++b;
    } else if (x < y) {
      ++a;
    } else {
      ++b;
    }
  }
  return c;
}

// Row i's set is counted into cnt[i] and kept in tmp[i * cap ...]; a copy
// kernel then packs it into P once the row pointers are known.
__global__ void k_interp_pattern(int n, int nx, int ny, int gkind, int geometric, int cap,
                                 const int *__restrict__ cf, const int *__restrict__ cidx,
                                 const int *__restrict__ grp, const int *__restrict__ gci,
                                 int *__restrict__ cnt, int *__restrict__ tmp) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int out[16];
  int m = 0;
  if (cf[i]) {
    out[m++] = cidx[i];
  } else if (geometric && gkind == 2) {
    const int ix = i % nx, iy = i / nx;
    for (int dy = -1; dy <= 1; ++dy)
      for (int dx = -1; dx <= 1; ++dx) {
        const int jx = ix + dx, jy = iy + dy;
        if (jx < 0 || jy < 0 || jx >= nx || jy >= ny) continue;
        const int j = jy * nx + jx;
        if (cf[j] && m < cap) out[m++] = cidx[j];
      }
  } else if (geometric && gkind == 1) {
    if (i - 1 >= 0 && cf[i - 1] && m < cap) out[m++] = cidx[i - 1];
    if (i + 1 < n && cf[i + 1] && m < cap) out[m++] = cidx[i + 1];
  } else {
    // keep the best `cap` candidates in a small array sorted by (score desc, j asc)
    int bj[16], bs[16];
    int nb = 0;
    for (int k = grp[i]; k < grp[i + 1]; ++k) {
      const int j = gci[k];
      if (!cf[j]) continue;
      const int sc = common_neighbours(grp, gci, i, j);
      // insertion: j ascending within equal scores holds because neighbours
      // are visited in ascending j and ties do not displace earlier entries
      int pos = nb;
      while (pos > 0 && bs[pos - 1] < sc) --pos;
      if (pos >= cap) continue;
      const int last = nb < cap ? nb : cap - 1;
      for (int q = last; q > pos; --q) {
        bj[q] = bj[q - 1];
        bs[q] = bs[q - 1];
      }
      bj[pos] = j;
      bs[pos] = sc;
      if (nb < cap) ++nb;
    }
    for (int q = 0; q < nb; ++q) out[q] = cidx[bj[q]];
    m = nb;
    // ascending coarse index
    for (int p = 1; p < m; ++p) {
      const int v = out[p];
      int q = p - 1;
      while (q >= 0 && out[q] > v) {
        out[q + 1] = out[q];
        --q;
      }
      out[q + 1] = v;
    }
  }
  cnt[i] = m;
  for (int q = 0; q < m; ++q) tmp[(size_t)i * cap + q] = out[q];
}

// Algebraic J_i with a group of W lanes per row (same result as the
// thread-per-row code above). Row i's neighbour list is staged in LDS; each
// lane scores its share of the coarse neighbours j (ascending j within the
// lane) by looking every entry of row j up in the staged row (binary
// search), and keeps its own best kJCap by (score desc, j asc). The group's
// lists then go to LDS, where each entry's rank in the group's order is
// counted: entries ranked below cap are J_i, and since the coarse index
// increases with j, the position of an entry in row i of P is the number of
// selected entries with smaller j. Rows longer than kJRow score by the
// sorted merge instead of the LDS lookup.
constexpr int kJCap = 8, kJRow = 128, kJThreads = 256;

__device__ __forceinline__ bool jbeats(int s2, int j2, int s1, int j1) {
  return s2 > s1 || (s2 == s1 && j2 < j1);
}

template <int W>
__global__ void __launch_bounds__(kJThreads)
    k_interp_alg(int n, int cap, const int *__restrict__ cf, const int *__restrict__ cidx,
                 const int *__restrict__ grp, const int *__restrict__ gci, int *__restrict__ cnt,
                 int *__restrict__ tmp) {
  constexpr int G = kJThreads / W;
  __shared__ int rowbuf[G][kJRow];
  __shared__ int ls[G][W * kJCap], lj[G][W * kJCap], lr[G][W * kJCap];
  const int g = threadIdx.x / W, lane = threadIdx.x % W;
  const int row = blockIdx.x * G + g;
  const bool live = row < n && !cf[row];
  const int r0 = row < n ? grp[row] : 0, rlen = row < n ? grp[row + 1] - r0 : 0;
  const bool staged = rlen <= kJRow;
  if (live && staged)
    for (int q = lane; q < rlen; q += W) rowbuf[g][q] = gci[r0 + q];
  __syncthreads();
  // this lane's best kJCap candidates, (score desc, j asc)
  int bs[kJCap], bj[kJCap], nb = 0;
#pragma unroll
  for (int q = 0; q < kJCap; ++q) bs[q] = bj[q] = 0;
  if (live) {
    for (int k = lane; k < rlen; k += W) {
      const int j = gci[r0 + k];
      if (!cf[j]) continue;
      int sc = 0;
      if (staged) {
        for (int b = grp[j]; b < grp[j + 1]; ++b) {
          const int v = gci[b];
          int lo = 0, hi = rlen;  // first position with rowbuf >= v
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (rowbuf[g][mid] < v)
              lo = mid + 1;
            else
              hi = mid;
          }
          sc += (lo < rlen && rowbuf[g][lo] == v) ? 1 : 0;
        }
      } else {
        sc = common_neighbours(grp, gci, row, j);
      }
      int pos = 0;  // entries ahead of (sc, j); j is the largest so far, so ties stay ahead
#pragma unroll
      for (int q = 0; q < kJCap; ++q) pos += (q < nb && bs[q] >= sc) ? 1 : 0;
      if (pos >= cap) continue;
#pragma unroll
      for (int q = kJCap - 1; q > 0; --q)
        if (q > pos && q < cap) {
          bs[q] = bs[q - 1];
          bj[q] = bj[q - 1];
        }
#pragma unroll
      for (int q = 0; q < kJCap; ++q)
        if (q == pos) {
          bs[q] = sc;
          bj[q] = j;
        }
      if (nb < cap) ++nb;
    }
  }
  // publish the lane's list (score -1 marks an empty slot)
#pragma unroll
  for (int q = 0; q < kJCap; ++q) {
    ls[g][lane * kJCap + q] = q < nb ? bs[q] : -1;
    lj[g][lane * kJCap + q] = bj[q];
  }
  __syncthreads();
  // rank of each own entry among the group's entries
  int rk[kJCap];
#pragma unroll
  for (int q = 0; q < kJCap; ++q) {
    rk[q] = 0;
    if (q >= nb) continue;
    for (int e = 0; e < W * kJCap; ++e) {
      const int s2 = ls[g][e];
      if (s2 >= 0 && jbeats(s2, lj[g][e], bs[q], bj[q])) ++rk[q];
    }
  }
#pragma unroll
  for (int q = 0; q < kJCap; ++q) lr[g][lane * kJCap + q] = q < nb ? rk[q] : 0x7fffffff;
  __syncthreads();
  if (row >= n) return;
  if (cf[row]) {
    if (lane == 0) {
      cnt[row] = 1;
      tmp[(size_t)row * cap] = cidx[row];
    }
    return;
  }
  int total = 0;  // group entries, computed by every lane alike
  for (int e = 0; e < W * kJCap; ++e) total += ls[g][e] >= 0 ? 1 : 0;
  if (lane == 0) cnt[row] = total < cap ? total : cap;
#pragma unroll
  for (int q = 0; q < kJCap; ++q) {
    if (q >= nb || rk[q] >= cap) continue;
    int p = 0;
    for (int e = 0; e < W * kJCap; ++e)
      if (lr[g][e] < cap && lj[g][e] < bj[q]) ++p;
    tmp[(size_t)row * cap + p] = cidx[bj[q]];
  }
}

__global__ void k_pack_rows(int n, int cap, const int *__restrict__ tmp,
                            const int *__restrict__ prp, int *__restrict__ pci) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int p0 = prp[i], m = prp[i + 1] - p0;
  for (int q = 0; q < m; ++q) pci[p0 + q] = tmp[(size_t)i * cap + q];
}

void interp_pattern(Pool &pool, const Level &L, int cap, int geometric, Csr &P, hipStream_t s) {
  const int n = L.n;
  if (cap > 16) fail(BAMG_E_ARG, "max_interp above 16");
  int *cnt = pool.get<int>(n);
  int *tmp = pool.get<int>((size_t)n * cap);
  if (!geometric && cap <= kJCap) {
    // lanes per row: the average row length of G, 8 to 64
    const int w = std::max(8, std::min(64, lanes_for(L.G.nr, L.G.nnz)));
    const int groups = kJThreads / w;
    switch (w) {
      case 8:
        k_interp_alg<8><<<ceil_div(n, groups), kJThreads, 0, s>>>(n, cap, L.cf, L.cidx, L.G.rp,
                                                                  L.G.ci, cnt, tmp);
        break;
      case 16:
        k_interp_alg<16><<<ceil_div(n, groups), kJThreads, 0, s>>>(n, cap, L.cf, L.cidx, L.G.rp,
                                                                   L.G.ci, cnt, tmp);
        break;
      case 32:
        k_interp_alg<32><<<ceil_div(n, groups), kJThreads, 0, s>>>(n, cap, L.cf, L.cidx, L.G.rp,
                                                                   L.G.ci, cnt, tmp);
        break;
      default:
        k_interp_alg<64><<<ceil_div(n, groups), kJThreads, 0, s>>>(n, cap, L.cf, L.cidx, L.G.rp,
                                                                   L.G.ci, cnt, tmp);
        break;
    }
  } else {
    k_interp_pattern<<<ceil_div(n, 128), 128, 0, s>>>(n, L.nx, L.ny, L.gkind, geometric, cap,
                                                       L.cf, L.cidx, L.G.rp, L.G.ci, cnt, tmp);
  }
  LAUNCHCHK();
  P.nr = n;
  P.nc = L.nc;
  P.rp = pool.get<int>(n + 1);
  scan_counts(pool, cnt, P.rp, n, s);
  P.nnz = read_int(P.rp + n, s);
  P.ci = pool.get<int>(P.nnz);
  k_pack_rows<<<ceil_div(n, 256), 256, 0, s>>>(n, cap, tmp, P.rp, P.ci);
  LAUNCHCHK();
  pool.release(cnt);
  pool.release(tmp);
}

// ============================================================ SpGEMM symbolic
// Rows of C = A * B with many product terms: one wave (block of 64) per
// listed row at a time. When the row's columns lie within kSymBitWords * 32
// of each other (the usual case for Galerkin rows), every term sets its
// column's bit in an LDS bitmap and the set bits are read back in order
// (k_spgemm_sym_narrow, which needs 1 KB of LDS, so many waves stay
// resident per CU); the other rows are listed again for k_spgemm_sym_wide,
// where every term appends its column to an LDS buffer, which is
// bitonic-sorted. The distinct columns are counted (pass 1) or written
// (pass 2). The result is the sorted structural product, independent of
// thread timing.
constexpr int kSymCap = 4096, kSymListBlocks = 4096, kSymNarrowBlocks = 8192;
constexpr int kSymBitWords = 256;

// The number of listed rows is read on the device (nlist), so the host does
// not wait for it: the grid strides over the list. Pass 1 appends the rows
// too wide for the bitmap to wide / nwide; pass 2 skips them.
template <bool FILL>
__global__ void __launch_bounds__(64)
    k_spgemm_sym_narrow(const int *__restrict__ rows, const int *__restrict__ nlist,
                        const int *__restrict__ arp, const int *__restrict__ aci,
                        const int *__restrict__ brp, const int *__restrict__ bci, int force_diag,
                        int *__restrict__ cnt, const int *__restrict__ crp,
                        int *__restrict__ cci, int *__restrict__ wide, int *__restrict__ nwide) {
  __shared__ unsigned bits[kSymBitWords];
  const int nl = *nlist, lane = threadIdx.x;
  for (int li = blockIdx.x; li < nl; li += gridDim.x) {
    const int row = rows[li];
    const int ab = arp[row], ae = arp[row + 1];
    // column span of the row's terms: rows of B are sorted, so each term
    // block contributes its first and last column
    int lo = force_diag ? row : 0x7fffffff, hi = force_diag ? row : -1;
    for (int a = ab + lane; a < ae; a += 64) {
      const int k = aci[a], b0 = brp[k], b1 = brp[k + 1];
      if (b1 > b0) {
        lo = min(lo, bci[b0]);
        hi = max(hi, bci[b1 - 1]);
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      lo = min(lo, __shfl_xor(lo, off, 64));
      hi = max(hi, __shfl_xor(hi, off, 64));
    }
    const int words = hi >= lo ? ((hi - lo) >> 5) + 1 : 0;
    if (words > kSymBitWords) {  // the same decision in both passes
      if (!FILL && lane == 0) wide[atomicAdd(nwide, 1)] = row;
      continue;
    }
    for (int q = lane; q < words; q += 64) bits[q] = 0u;
    __syncthreads();
    if (force_diag && lane == 0) atomicOr(&bits[(row - lo) >> 5], 1u << ((row - lo) & 31));
    for (int a = ab + lane; a < ae; a += 64) {
      const int k = aci[a];
      for (int b = brp[k]; b < brp[k + 1]; ++b) {
        const int d = bci[b] - lo;
        atomicOr(&bits[d >> 5], 1u << (d & 31));
      }
    }
    __syncthreads();
    int base = 0;
    const int out0 = FILL ? crp[row] : 0;
    for (int q0 = 0; q0 < words; q0 += 64) {
      const int q = q0 + lane;
      const unsigned wbits = q < words ? bits[q] : 0u;
      // exclusive prefix of the popcounts over the wave
      int c = __popc(wbits), incl = c;
      for (int off = 1; off < 64; off <<= 1) {
        const int v = __shfl_up(incl, off, 64);
        if (lane >= off) incl += v;
      }
      if (FILL) {
        unsigned m = wbits;
        int o = out0 + base + incl - c;
        while (m) {
          const int bb = __ffs(m) - 1;
          cci[o++] = lo + (q << 5) + bb;
          m &= m - 1;
        }
      }
      base += __shfl(incl, 63, 64);
    }
    if (!FILL && lane == 0) cnt[row] = base;
    __syncthreads();  // bits is reused by the next listed row
  }
}

template <bool FILL>
__global__ void __launch_bounds__(64)
    k_spgemm_sym_wide(const int *__restrict__ rows, const int *__restrict__ nlist,
                      const int *__restrict__ arp, const int *__restrict__ aci,
                      const int *__restrict__ brp, const int *__restrict__ bci, int force_diag,
                      int *__restrict__ cnt, const int *__restrict__ crp, int *__restrict__ cci,
                      int *__restrict__ overflow) {
  __shared__ int buf[kSymCap];
  __shared__ int nbuf;
  const int nl = *nlist, lane = threadIdx.x;
  for (int li = blockIdx.x; li < nl; li += gridDim.x) {
    const int row = rows[li];
    const int ab = arp[row], ae = arp[row + 1];
    // gather the terms and sort them
    if (lane == 0) nbuf = 0;
    __syncthreads();
    if (force_diag && lane == 0) {
      buf[0] = row;
      nbuf = 1;
    }
    __syncthreads();
    for (int a = ab + lane; a < ae; a += 64) {
      const int k = aci[a];
      for (int b = brp[k]; b < brp[k + 1]; ++b) {
        const int pos = atomicAdd(&nbuf, 1);
        if (pos < kSymCap) buf[pos] = bci[b];
      }
    }
    __syncthreads();
    int cntv = nbuf;
    if (cntv > kSymCap) {
      if (lane == 0) atomicOr(overflow, 1);
      cntv = kSymCap;
    }
    int P2 = 1;
    while (P2 < cntv) P2 <<= 1;
    for (int i = cntv + lane; i < P2; i += 64) buf[i] = 0x7fffffff;
    __syncthreads();
    // bitonic sort of buf[0..P2)
    for (int size = 2; size <= P2; size <<= 1) {
      for (int stride = size >> 1; stride > 0; stride >>= 1) {
        for (int i = lane; i < (P2 >> 1); i += 64) {
          const int lo = 2 * i - (i & (stride - 1));
          const int hi = lo + stride;
          const bool up = (lo & size) == 0;
          const int x = buf[lo], y = buf[hi];
          if ((x > y) == up) {
            buf[lo] = y;
            buf[hi] = x;
          }
        }
        __syncthreads();
      }
    }
    // distinct values, written in order with a running count per 64-chunk
    int base = 0;
    const int out0 = FILL ? crp[row] : 0;
    for (int c0 = 0; c0 < cntv; c0 += 64) {
      const int i = c0 + lane;
      const bool isnew = i < cntv && (i == 0 || buf[i] != buf[i - 1]);
      const uint64_t mask = __ballot(isnew);
      const int before = __popcll(mask & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
      if (FILL && isnew) cci[out0 + base + before] = buf[i];
      base += __popcll(mask);
    }
    if (!FILL && lane == 0) cnt[row] = base;
    __syncthreads();  // buf and nbuf are reused by the next listed row
  }
}

// Short rows (at most kSymShort candidate terms, the common case of the
// Galerkin products): one thread per row sorts its candidates in a private
// LDS slice (position-major) and counts or writes the distinct columns.
// Longer rows are listed for the wave-per-row kernel above (rowlist).
constexpr int kSymShort = 32, kSymThreads = 128;

// The distinct columns of each short row are kept in tmp[row * kSymShort ..]
// (counted into cnt) and packed into C by k_sym_pack once C's row pointers
// are known; a long row has tmp[row * kSymShort] = -1.
__global__ void __launch_bounds__(kSymThreads)
    k_spgemm_sym_short(int nr, const int *__restrict__ arp, const int *__restrict__ aci,
                       const int *__restrict__ brp, const int *__restrict__ bci, int force_diag,
                       int *__restrict__ cnt, int *__restrict__ tmp, int *__restrict__ longrows,
                       int *__restrict__ nlong) {
  __shared__ int buf[kSymShort * kSymThreads];
  const int t = threadIdx.x;
  const int row = blockIdx.x * kSymThreads + t;
  bool is_long = false;
  if (row < nr) {
    int total = force_diag ? 1 : 0;
    for (int a = arp[row]; a < arp[row + 1]; ++a) total += brp[aci[a] + 1] - brp[aci[a]];
    if (total > kSymShort) {
      is_long = true;
      tmp[(size_t)row * kSymShort] = -1;  // written by the list kernel instead
    } else {
      int m = 0;
      if (force_diag) buf[(m++) * kSymThreads + t] = row;
      for (int a = arp[row]; a < arp[row + 1]; ++a) {
        const int k = aci[a];
        for (int b = brp[k]; b < brp[k + 1]; ++b) {
          // insertion into the sorted slice
          const int v = bci[b];
          int q = m++;
          while (q > 0 && buf[(q - 1) * kSymThreads + t] > v) {
            buf[q * kSymThreads + t] = buf[(q - 1) * kSymThreads + t];
            --q;
          }
          buf[q * kSymThreads + t] = v;
        }
      }
      int d = 0;
      for (int q = 0; q < m; ++q) {
        const int v = buf[q * kSymThreads + t];
        if (q == 0 || v != buf[(q - 1) * kSymThreads + t]) tmp[(size_t)row * kSymShort + d++] = v;
      }
      cnt[row] = d;
    }
  }
  const unsigned long long bl = __ballot(is_long);
  if (bl) {
    int base = 0;
    if ((t % kWave) == 0) base = atomicAdd(nlong, (int)__popcll(bl));
    base = __shfl(base, 0, kWave);
    const int lane = t % kWave;
    if (is_long) longrows[base + __popcll(bl & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))))] = row;
  }
}

__global__ void k_sym_pack(int nr, const int *__restrict__ tmp,
                           const int *__restrict__ crp, int *__restrict__ cci) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nr) return;
  const int p0 = crp[i], m = crp[i + 1] - p0;
  if (m == 0 || tmp[(size_t)i * kSymShort] < 0) return;  // long rows: the list kernel
  for (int q = 0; q < m; ++q) cci[p0 + q] = tmp[(size_t)i * kSymShort + q];
}

// Symbolic product in two halves, so that two independent products share
// one host round trip: the count half enqueues the row counts, the scan and
// the copies of the size and the overflow flag to the host; the finish half
// (after the caller has synchronised s) allocates the column indices and
// enqueues the packing.
struct SymJob {
  const Csr *A = nullptr, *B = nullptr;
  int force_diag = 0, lgrid = 0;
  Csr *C = nullptr;
  int *cnt = nullptr, *tmp = nullptr, *ovf = nullptr, *longrows = nullptr, *widerows = nullptr;
  int *hv = nullptr;  // pinned: C's size and the overflow flag, copied by the count half
};

static void sym_count(Pool &pool, const Csr &A, const Csr &B, int force_diag, Csr &C, SymJob &j,
                      int *hv, hipStream_t s) {
  const int nr = A.nr;
  j.hv = hv;
  j.A = &A;
  j.B = &B;
  j.force_diag = force_diag;
  j.C = &C;
  j.cnt = pool.get<int>(nr);
  j.tmp = pool.get<int>((size_t)nr * kSymShort);
  j.ovf = pool.get<int>(3);  // [overflow, long rows, wide rows]
  j.longrows = pool.get<int>(nr);
  j.widerows = pool.get<int>(nr);
  fill_i32(j.ovf, 0, 3, s);
  if (nr) {
    k_spgemm_sym_short<<<ceil_div(nr, kSymThreads), kSymThreads, 0, s>>>(
        nr, A.rp, A.ci, B.rp, B.ci, force_diag, j.cnt, j.tmp, j.longrows, j.ovf + 1);
    LAUNCHCHK();
  }
  // long rows: strided grids about as wide as the LDS lets stay resident
  j.lgrid = std::min(nr, kSymListBlocks);
  if (j.lgrid > 0) {
    k_spgemm_sym_narrow<false><<<std::min(nr, kSymNarrowBlocks), 64, 0, s>>>(
        j.longrows, j.ovf + 1, A.rp, A.ci, B.rp, B.ci, force_diag, j.cnt, nullptr, nullptr,
        j.widerows, j.ovf + 2);
    LAUNCHCHK();
    k_spgemm_sym_wide<false><<<j.lgrid, 64, 0, s>>>(j.widerows, j.ovf + 2, A.rp, A.ci, B.rp,
                                                    B.ci, force_diag, j.cnt, nullptr, nullptr,
                                                    j.ovf);
    LAUNCHCHK();
  }
  C.nr = nr;
  C.nc = B.nc;
  C.rp = pool.get<int>(nr + 1);
  scan_counts(pool, j.cnt, C.rp, nr, s);
  HIPCHK(hipMemcpyAsync(&j.hv[0], C.rp + nr, sizeof(int), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemcpyAsync(&j.hv[1], j.ovf, sizeof(int), hipMemcpyDeviceToHost, s));
}

static void sym_finish(Pool &pool, SymJob &j, hipStream_t s) {
  const Csr &A = *j.A, &B = *j.B;
  Csr &C = *j.C;
  const int nr = A.nr;
  if (j.hv[1]) fail(BAMG_E_ARG, "Galerkin row wider than the symbolic buffer");
  C.nnz = j.hv[0];
  C.ci = pool.get<int>(C.nnz);
  if (nr) {
    k_sym_pack<<<ceil_div(nr, 256), 256, 0, s>>>(nr, j.tmp, C.rp, C.ci);
    LAUNCHCHK();
  }
  if (j.lgrid > 0) {
    k_spgemm_sym_narrow<true><<<std::min(nr, kSymNarrowBlocks), 64, 0, s>>>(
        j.longrows, j.ovf + 1, A.rp, A.ci, B.rp, B.ci, j.force_diag, nullptr, C.rp, C.ci,
        nullptr, nullptr);
    LAUNCHCHK();
    k_spgemm_sym_wide<true><<<j.lgrid, 64, 0, s>>>(j.widerows, j.ovf + 2, A.rp, A.ci, B.rp, B.ci,
                                                   j.force_diag, nullptr, C.rp, C.ci, j.ovf);
    LAUNCHCHK();
  }
  pool.release(j.cnt);
  pool.release(j.tmp);
  pool.release(j.ovf);
  pool.release(j.longrows);
  pool.release(j.widerows);
}

void spgemm_symbolic2(Pool &pool, const Csr &A1, const Csr &B1, const Csr &A2, const Csr &B2,
                      int force_diag, Csr &C1, Csr &C2, hipStream_t s) {
  SymJob j1, j2;
  int *hv = pool.pinned();
  sym_count(pool, A1, B1, force_diag, C1, j1, hv, s);
  sym_count(pool, A2, B2, force_diag, C2, j2, hv + 2, s);
  HIPCHK(hipStreamSynchronize(s));
  sym_finish(pool, j1, s);
  sym_finish(pool, j2, s);
}

// ============================================================ SpGEMM numeric
// One thread per row of C: terms are added in the order (A column, B column)
// ascending, each at the position of its column in the sorted row of C.
// Rows of C with at most kNumAcc entries and kNumTerms product terms
// accumulate in the thread's private LDS slice, next to the row's column
// indices that the binary search reads (both laid out position-major so
// the threads of a wave hit distinct banks) and are written once.
constexpr int kNumThreads = 128, kNumAcc = 32, kNumTerms = 64;

template <class T>
__global__ void __launch_bounds__(kNumThreads)
    k_spgemm_num_lds(int nr, const int *__restrict__ arp, const int *__restrict__ aci,
                     const T *__restrict__ av, const int *__restrict__ brp,
                     const int *__restrict__ bci, const T *__restrict__ bv,
                     const int *__restrict__ crp, const int *__restrict__ cci,
                     T *__restrict__ cv, int *__restrict__ longrows, int *__restrict__ nlong) {
  __shared__ T acc[kNumAcc * kNumThreads];
  __shared__ int cols[kNumAcc * kNumThreads];  // the output row's columns
  const int t = threadIdx.x;
  const int i = blockIdx.x * kNumThreads + t;
  bool is_long = false;
  if (i < nr) {
    const int c0 = crp[i], c1 = crp[i + 1];
    const int m = c1 - c0;
    int terms = 0;
    for (int a = arp[i]; a < arp[i + 1] && terms <= kNumTerms; ++a)
      terms += brp[aci[a] + 1] - brp[aci[a]];
    if (m > kNumAcc || terms > kNumTerms) {
      is_long = true;
    } else {
      for (int q = 0; q < m; ++q) {
        acc[q * kNumThreads + t] = (T)0;
        cols[q * kNumThreads + t] = cci[c0 + q];
      }
      for (int a = arp[i]; a < arp[i + 1]; ++a) {
        const int k = aci[a];
        const T x = av[a];
        for (int b = brp[k]; b < brp[k + 1]; ++b) {
          const int j = bci[b];
          int lo = 0, hi = m - 1;
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (cols[mid * kNumThreads + t] < j)
              lo = mid + 1;
            else
              hi = mid;
          }
          acc[lo * kNumThreads + t] += x * bv[b];
        }
      }
      for (int q = 0; q < m; ++q) cv[c0 + q] = acc[q * kNumThreads + t];
    }
  }
  // rows with more than kNumAcc entries or kNumTerms product terms go to
  // k_spgemm_num_long (one counter update per wave)
  const unsigned long long bl = __ballot(is_long);
  if (bl) {
    const int lane = t % kWave;
    int base = 0;
    if (lane == 0) base = atomicAdd(nlong, (int)__popcll(bl));
    base = __shfl(base, 0, kWave);
    if (is_long) longrows[base + __popcll(bl & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))))] = i;
  }
}

// Long rows of C: a group of kLongLanes lanes per row. Lane l takes a
// contiguous chunk of the row of A and accumulates its terms into its own
// LDS slice; the slices are then summed in lane order, so the result does
// not depend on timing. Rows wider than kLongAcc are summed by one lane in
// global memory.
constexpr int kLongLanes = 16, kLongGroups = 4, kLongAcc = 96, kNumFewRows = 32768;

template <class T>
__global__ void __launch_bounds__(kLongLanes * kLongGroups)
    k_spgemm_num_long(const int *__restrict__ rows, const int *__restrict__ nlong, int nall,
                      const int *__restrict__ arp, const int *__restrict__ aci,
                      const T *__restrict__ av, const int *__restrict__ brp,
                      const int *__restrict__ bci, const T *__restrict__ bv,
                      const int *__restrict__ crp, const int *__restrict__ cci,
                      T *__restrict__ cv) {
  __shared__ T acc[kLongGroups][kLongAcc * kLongLanes];
  __shared__ int cols[kLongGroups][kLongAcc];
  const int g = threadIdx.x / kLongLanes, lane = threadIdx.x % kLongLanes;
  const int nl = rows ? *nlong : nall;  // rows == nullptr: every row of C
  for (int base = blockIdx.x * kLongGroups; base < nl; base += gridDim.x * kLongGroups) {
    const int w = base + g;
    const int i = w < nl ? (rows ? rows[w] : w) : -1;
    const int c0 = i >= 0 ? crp[i] : 0, m = i >= 0 ? crp[i + 1] - c0 : 0;
    const bool lds = m <= kLongAcc;
    if (i >= 0 && lds) {
      for (int q = lane; q < m; q += kLongLanes) cols[g][q] = cci[c0 + q];
      for (int q = 0; q < m; ++q) acc[g][q * kLongLanes + lane] = (T)0;
    }
    __syncthreads();
    if (i >= 0 && lds) {
      const int ab = arp[i], ae = arp[i + 1];
      const int chunk = (ae - ab + kLongLanes - 1) / kLongLanes;
      const int a1 = ab + lane * chunk, a2 = min(ae, a1 + chunk);
      for (int a = a1; a < a2; ++a) {
        const int k = aci[a];
        const T x = av[a];
        for (int b = brp[k]; b < brp[k + 1]; ++b) {
          const int j = bci[b];
          int lo = 0, hi = m - 1;
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (cols[g][mid] < j)
              lo = mid + 1;
            else
              hi = mid;
          }
          acc[g][lo * kLongLanes + lane] += x * bv[b];
        }
      }
    } else if (i >= 0 && lane == 0) {
      for (int p = c0; p < c0 + m; ++p) cv[p] = (T)0;
      for (int a = arp[i]; a < arp[i + 1]; ++a) {
        const int k = aci[a];
        const T x = av[a];
        for (int b = brp[k]; b < brp[k + 1]; ++b) {
          const int j = bci[b];
          int lo = c0, hi = c0 + m - 1;
          while (lo < hi) {
            const int mid = (lo + hi) >> 1;
            if (cci[mid] < j)
              lo = mid + 1;
            else
              hi = mid;
          }
          cv[lo] += x * bv[b];
        }
      }
    }
    __syncthreads();
    if (i >= 0 && lds)
      for (int q = lane; q < m; q += kLongLanes) {
        T sum = (T)0;
        for (int l = 0; l < kLongLanes; ++l) sum += acc[g][q * kLongLanes + l];
        cv[c0 + q] = sum;
      }
    __syncthreads();
  }
}

template <class T>
void spgemm_numeric(const Csr &A, const T *av, const Csr &B, const T *bv, const Csr &C, T *cv,
                    int *scratch, hipStream_t s) {
  if (!A.nr) return;
  const int grid = std::min(1024, ceil_div(A.nr, kLongGroups));
  if (A.nr < kNumFewRows) {
    // few rows: a thread per row cannot hide its chain of dependent loads,
    // so every row goes to the lane groups
    k_spgemm_num_long<T><<<grid, kLongLanes * kLongGroups, 0, s>>>(
        nullptr, nullptr, A.nr, A.rp, A.ci, av, B.rp, B.ci, bv, C.rp, C.ci, cv);
    LAUNCHCHK();
    return;
  }
  int *nlong = scratch, *longrows = scratch + 1;  // scratch holds A.nr + 1 ints
  fill_i32(nlong, 0, 1, s);
  k_spgemm_num_lds<T><<<ceil_div(A.nr, kNumThreads), kNumThreads, 0, s>>>(
      A.nr, A.rp, A.ci, av, B.rp, B.ci, bv, C.rp, C.ci, cv, longrows, nlong);
  LAUNCHCHK();
  k_spgemm_num_long<T><<<grid, kLongLanes * kLongGroups, 0, s>>>(
      longrows, nlong, 0, A.rp, A.ci, av, B.rp, B.ci, bv, C.rp, C.ci, cv);
  LAUNCHCHK();
}

// ============================================================ LS fits
// Array bounds of one fit: RM test vectors, MM interpolation points. The
// small instance (RM = 8, MM = 4, the paper's r = 8 with c <= 4) keeps its
// arrays in registers; the large one (16, 8) covers the remaining options.
constexpr int kRMax = 16, kMMax = 8;

// Every array below is indexed only by loop counters of fully unrolled
// loops over the compile-time bounds RM, MM (rows and points beyond the
// live counts are masked off), so the compiler keeps the arrays in
// registers. Point sets are bitmasks over the MM positions; a column's
// place in the factorisation is its rank among the set bits.

// Householder least squares over the point set `mask`: minimise
// || W[:, mask] p - h || over rows [0, nrow), W and h produced by
// build(W, h) (rows >= nrow zero). Columns enter in increasing position;
// column t eliminates at pivot row rank(t). Only the first nrow columns can
// be determined (the rest are dropped), and a column whose |R_tt| falls to
// 1e-12 max |R_ss| or below is dropped; after a drop the fit is redone from
// build(). Returns the set kept, with p[t] for its positions.
template <int RM, int MM, class Build>
__device__ unsigned ls_qr(Build build, int nrow, unsigned mask, double (&p)[MM]) {
  for (;;) {
    if (mask == 0) return 0;
    double W[RM][MM], h[RM], R[MM];
    build(W, h);
    const int na = __popc(mask);
    int a = 0;  // pivot row of the next column
#pragma unroll
    for (int t = 0; t < MM; ++t) {
      R[t] = 0.0;
      if (!((mask >> t) & 1u) || a >= nrow) continue;
      double nrm = 0.0, x0 = 0.0;
#pragma unroll
      for (int k = 0; k < RM; ++k)
        if (k >= a && k < nrow) nrm += W[k][t] * W[k][t];
      nrm = sqrt(nrm);
#pragma unroll
      for (int k = 0; k < RM; ++k)
        if (k == a) x0 = W[k][t];
      const double alpha = x0 >= 0 ? -nrm : nrm;
      R[t] = alpha;
      if (nrm != 0.0) {
#pragma unroll
        for (int k = 0; k < RM; ++k)
          if (k == a) W[k][t] = x0 - alpha;
        double vtv = 0.0;
#pragma unroll
        for (int k = 0; k < RM; ++k)
          if (k >= a && k < nrow) vtv += W[k][t] * W[k][t];
        if (vtv != 0.0) {
#pragma unroll
          for (int b = t + 1; b < MM; ++b) {
            if (!((mask >> b) & 1u)) continue;
            double sb = 0.0;
#pragma unroll
            for (int k = 0; k < RM; ++k)
              if (k >= a && k < nrow) sb += W[k][t] * W[k][b];
            sb = 2.0 * sb / vtv;
#pragma unroll
            for (int k = 0; k < RM; ++k)
              if (k >= a && k < nrow) W[k][b] -= sb * W[k][t];
          }
          double sh = 0.0;
#pragma unroll
          for (int k = 0; k < RM; ++k)
            if (k >= a && k < nrow) sh += W[k][t] * h[k];
          sh = 2.0 * sh / vtv;
#pragma unroll
          for (int k = 0; k < RM; ++k)
            if (k >= a && k < nrow) h[k] -= sh * W[k][t];
        }
      }
      ++a;
    }
    if (na > nrow) {
      // keep the first nrow columns
      unsigned keep = 0;
      int cnt = 0;
#pragma unroll
      for (int t = 0; t < MM; ++t)
        if ((mask >> t) & 1u) {
          if (cnt < nrow) keep |= 1u << t;
          ++cnt;
        }
      mask = keep;
      continue;
    }
    double rmax = 0.0;
#pragma unroll
    for (int t = 0; t < MM; ++t)
      if ((mask >> t) & 1u) rmax = fmax(rmax, fabs(R[t]));
    int drop = -1;
#pragma unroll
    for (int t = 0; t < MM; ++t)
      if (drop < 0 && ((mask >> t) & 1u) && !(fabs(R[t]) > 1e-12 * rmax)) drop = t;
    if (drop >= 0) {
      mask &= ~(1u << drop);
      continue;
    }
    // back substitution, last column first; column t's pivot row is rank(t)
#pragma unroll
    for (int t = MM - 1; t >= 0; --t) {
      if (!((mask >> t) & 1u)) continue;
      const int at = __popc(mask & ((1u << t) - 1u));
      double sum = 0.0;
#pragma unroll
      for (int k = 0; k < RM; ++k)
        if (k == at) sum = h[k];
#pragma unroll
      for (int b = t + 1; b < MM; ++b) {
        if (!((mask >> b) & 1u)) continue;
        double wab = 0.0;
#pragma unroll
        for (int k = 0; k < RM; ++k)
          if (k == at) wab = W[k][b];
        sum -= wab * p[b];
      }
      p[t] = sum / R[t];
    }
    return mask;
  }
}

// One weighted fit over the point set act (bits < m): plain (sum1 = false,
// rows k = 0..r-1) or with sum-to-one (rows k = 1..r-1, the highest active
// point eliminated). Writes coef[0..MM) (0 for points outside the set).
template <int RM, int MM>
__device__ void fit_active(const double (&Gr)[RM][MM], const double (&gr)[RM],
                           const double *__restrict__ w, int r, bool sum1, unsigned act,
                           double (&coef)[MM]) {
  double p[MM];
#pragma unroll
  for (int t = 0; t < MM; ++t) {
    coef[t] = 0.0;
    p[t] = 0.0;
  }
  if (act == 0) return;
  if (!sum1) {
    auto build = [&](double (&W)[RM][MM], double (&h)[RM]) {
#pragma unroll
      for (int k = 0; k < RM; ++k) {
        const double sw = k < r ? sqrt(w[k]) : 0.0;
#pragma unroll
        for (int t = 0; t < MM; ++t) W[k][t] = sw * Gr[k][t];
        h[k] = sw * gr[k];
      }
    };
    const unsigned kept = ls_qr<RM, MM>(build, r, act, p);
#pragma unroll
    for (int t = 0; t < MM; ++t)
      if ((kept >> t) & 1u) coef[t] = p[t];
    return;
  }
  const int last = 31 - __clz(act);
  if (act == (1u << last)) {
    coef[last] = 1.0;
    return;
  }
  double glast[RM];
#pragma unroll
  for (int k = 0; k < RM; ++k) {
    glast[k] = 0.0;
#pragma unroll
    for (int t = 0; t < MM; ++t)
      if (t == last) glast[k] = Gr[k][t];
  }
  // row k' of the fit is row k' + 1 of the test vectors
  auto build = [&](double (&W)[RM][MM], double (&h)[RM]) {
#pragma unroll
    for (int kk = 0; kk < RM; ++kk) {
      const int k = kk + 1;
      if (k < RM && k < r) {
        const double sw = sqrt(w[k]);
        const double lv = glast[k < RM ? k : 0];
#pragma unroll
        for (int t = 0; t < MM; ++t) W[kk][t] = sw * (Gr[k < RM ? k : 0][t] - lv);
        h[kk] = sw * (gr[k < RM ? k : 0] - lv);
      } else {
#pragma unroll
        for (int t = 0; t < MM; ++t) W[kk][t] = 0.0;
        h[kk] = 0.0;
      }
    }
  };
  const unsigned kept = ls_qr<RM, MM>(build, r - 1, act & ~(1u << last), p);
  double sum = 0.0;
#pragma unroll
  for (int t = 0; t < MM; ++t)
    if ((kept >> t) & 1u) {
      coef[t] = p[t];
      sum += p[t];
    }
#pragma unroll
  for (int t = 0; t < MM; ++t)
    if (t == last) coef[t] = 1.0 - sum;
}

// rule 1: while a weight is negative, remove the most negative point (the
// lowest position among equals) and refit (at least one point stays).
template <int RM, int MM>
__device__ void fit_point(const double (&G)[RM][MM], const double (&g)[RM],
                          const double *__restrict__ w, int r, int m, bool sum1, int rule,
                          double (&coef)[MM]) {
  unsigned act = (m >= 32) ? ~0u : ((1u << m) - 1u);
  for (;;) {
    fit_active<RM, MM>(G, g, w, r, sum1, act, coef);
    if (rule == 0 || __popc(act) == 1) return;
    int worst = -1;
    double cw = 0.0;
#pragma unroll
    for (int t = 0; t < MM; ++t)
      if (((act >> t) & 1u) && coef[t] < 0.0 && (worst < 0 || coef[t] < cw)) {
        worst = t;
        cw = coef[t];
      }
    if (worst < 0) return;
    act &= ~(1u << worst);
  }
}

template <class T, int RM, int MM>
__global__ void __launch_bounds__(64)
    k_ls_fit(int n, int r, const int *__restrict__ cf, const int *__restrict__ prp,
             const int *__restrict__ pci, const int *__restrict__ cpts, const T *__restrict__ U,
             const T *__restrict__ V, const double *__restrict__ wv,
             const double *__restrict__ wu, int rule, int average, T *__restrict__ Pv,
             T *__restrict__ Qtv) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int a0 = prp[i];
  if (cf[i]) {
    Pv[a0] = (T)1;
    Qtv[a0] = (T)1;
    return;
  }
  const int m = prp[i + 1] - a0;
  int jf[MM];
#pragma unroll
  for (int t = 0; t < MM; ++t) jf[t] = t < m ? cpts[pci[a0 + t]] : 0;
  double G[RM][MM], g[RM], coef[MM];
#pragma unroll
  for (int k = 0; k < RM; ++k) {
#pragma unroll
    for (int t = 0; t < MM; ++t) G[k][t] = (k < r && t < m) ? (double)V[(size_t)jf[t] * r + k] : 0.0;
    g[k] = k < r ? (double)V[(size_t)i * r + k] : 0.0;
  }
  fit_point<RM, MM>(G, g, wv, r, m, false, rule, coef);
#pragma unroll
  for (int t = 0; t < MM; ++t)
    if (t < m) Pv[a0 + t] = (T)coef[t];
  if (average) {
    // simple averaging (Section 5): every entry of column i of Q is 1 / |J_i|
    for (int t = 0; t < m; ++t) Qtv[a0 + t] = (T)(1.0 / m);
    return;
  }
#pragma unroll
  for (int k = 0; k < RM; ++k) {
#pragma unroll
    for (int t = 0; t < MM; ++t) G[k][t] = (k < r && t < m) ? (double)U[(size_t)jf[t] * r + k] : 0.0;
    g[k] = k < r ? (double)U[(size_t)i * r + k] : 0.0;
  }
  fit_point<RM, MM>(G, g, wu, r, m, true, rule, coef);
#pragma unroll
  for (int t = 0; t < MM; ++t)
    if (t < m) Qtv[a0 + t] = (T)coef[t];
}

template <class T>
void ls_fit(const Level &L, int r, int mmax, const T *U, const T *V, const double *wv,
            const double *wu, int rule, int average, T *Pv, T *Qtv, hipStream_t s) {
  if (r > kRMax) fail(BAMG_E_ARG, "r above 16");
  if (mmax > kMMax) fail(BAMG_E_ARG, "more than 8 interpolation points");
  if (r <= 8 && mmax <= 4)
    k_ls_fit<T, 8, 4><<<ceil_div(L.n, 64), 64, 0, s>>>(L.n, r, L.cf, L.P.rp, L.P.ci, L.cpts, U, V,
                                                      wv, wu, rule, average, Pv, Qtv);
  else
    k_ls_fit<T, kRMax, kMMax><<<ceil_div(L.n, 64), 64, 0, s>>>(L.n, r, L.cf, L.P.rp, L.P.ci, L.cpts,
                                                              U, V, wv, wu, rule, average, Pv,
                                                              Qtv);
  LAUNCHCHK();
}

template <class T>
__global__ void k_fill_transfer_identity(int n, const int *__restrict__ cf,
                                         const int *__restrict__ prp, T *__restrict__ Pv,
                                         T *__restrict__ Qtv) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int a0 = prp[i], m = prp[i + 1] - a0;
  for (int t = 0; t < m; ++t) {
    Pv[a0 + t] = cf[i] ? (T)1 : (T)(1.0 / m);
    Qtv[a0 + t] = cf[i] ? (T)1 : (T)(1.0 / m);
  }
}

template <class T>
void fill_transfer_identity(const Level &L, T *Pv, T *Qtv, hipStream_t s) {
  k_fill_transfer_identity<T><<<ceil_div(L.n, 256), 256, 0, s>>>(L.n, L.cf, L.P.rp, Pv, Qtv);
  LAUNCHCHK();
}

// ============================================================ small helpers
template <class T>
__global__ void k_dinv(int n, const int *__restrict__ dpos, const T *__restrict__ bv,
                       T *__restrict__ dinv, int *__restrict__ flag) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int p = dpos[i];
  const T d = p >= 0 ? bv[p] : (T)0;
  if (!(d != (T)0) || !isfinite((double)d)) {
    atomicOr(flag, 1);
    dinv[i] = (T)0;
  } else {
    dinv[i] = (T)1 / d;
  }
}

// check = false: the flag only accumulates (the caller zeroed it and reads
// it later, sparing a host round trip per level).
template <class T>
void dinv_from_diag(const Level &L, const T *bv, T *dinv, int *flag, bool check, hipStream_t s) {
  if (check) fill_i32(flag, 0, 1, s);
  k_dinv<T><<<ceil_div(L.n, 256), 256, 0, s>>>(L.n, L.dpos, bv, dinv, flag);
  LAUNCHCHK();
  if (check && read_int(flag, s))
    fail(BAMG_E_BAD_DIAG, "zero or non-finite diagonal in some B_l");
}

template <class T>
__global__ void k_inject(const int *__restrict__ cpts, int nc, int r, const T *__restrict__ X,
                         T *__restrict__ Xc) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)nc * r) return;
  const int a = (int)(idx / r), k = (int)(idx % r);
  Xc[idx] = X[(size_t)cpts[a] * r + k];
}

template <class T>
void inject(const int *cpts, int nc, int r, const T *X, T *Xc, hipStream_t s) {
  long tot = (long)nc * r;
  if (!tot) return;
  k_inject<T><<<ceil_div(tot, 256), 256, 0, s>>>(cpts, nc, r, X, Xc);
  LAUNCHCHK();
}

// Y = A X, r columns row-major; thread per (row, column)
template <class T>
__global__ void k_spmm(int nr, int r, const int *__restrict__ rp, const int *__restrict__ ci,
                       const T *__restrict__ av, const T *__restrict__ X, T *__restrict__ Y,
                       int reset0) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)nr * r) return;
  const int i = (int)(idx / r), k = (int)(idx % r);
  if (reset0 && k == 0) {
    Y[idx] = (T)1;
    return;
  }
  T s = 0;
  for (int a = rp[i]; a < rp[i + 1]; ++a) s += av[a] * X[(size_t)ci[a] * r + k];
  Y[idx] = s;
}

template <class T>
void spmm(const Csr &A, const T *av, int r, const T *X, T *Y, int reset0, hipStream_t s) {
  long tot = (long)A.nr * r;
  if (!tot) return;
  k_spmm<T><<<ceil_div(tot, 256), 256, 0, s>>>(A.nr, r, A.rp, A.ci, av, X, Y, reset0);
  LAUNCHCHK();
}

// ============================================================ relaxation
// sum over a in [a0, a1) of val[a] * X[ci[a] * r + k], in index order,
// accumulated in A. Four entries at a time: their indices, values and
// gathered vector entries are loaded before any product, so a thread keeps
// four independent loads in flight instead of one dependent chain.
template <class A, class T>
__device__ __forceinline__ A row_dot(int a0, int a1, const int *__restrict__ ci,
                                     const T *__restrict__ val, const T *__restrict__ X, int r,
                                     int k) {
  A acc = 0;
  int a = a0;
  for (; a + 4 <= a1; a += 4) {
    int c[4];
    T w[4], x[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      c[j] = ci[a + j];
      w[j] = val[a + j];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) x[j] = X[(size_t)c[j] * r + k];
#pragma unroll
    for (int j = 0; j < 4; ++j) acc += (A)w[j] * (A)x[j];
  }
  for (; a < a1; ++a) acc += (A)val[a] * (A)X[(size_t)ci[a] * r + k];
  return acc;
}

// The same for two value arrays on one pattern: (mv . U, nv . V) on row i
// of M (whose pattern N shares).
template <class A, class T>
__device__ __forceinline__ void row_dot2(int a0, int a1, const int *__restrict__ ci,
                                         const T *__restrict__ mv, const T *__restrict__ nv,
                                         const T *__restrict__ U, const T *__restrict__ V, int r,
                                         int k, A &mu, A &nvv) {
  mu = 0;
  nvv = 0;
  int a = a0;
  for (; a + 2 <= a1; a += 2) {
    const size_t j0 = (size_t)ci[a] * r + k, j1 = (size_t)ci[a + 1] * r + k;
    const T m0 = mv[a], m1 = mv[a + 1], n0 = nv[a], n1 = nv[a + 1];
    const T u0 = U[j0], u1 = U[j1], v0 = V[j0], v1 = V[j1];
    mu += (A)m0 * (A)u0;
    nvv += (A)n0 * (A)v0;
    mu += (A)m1 * (A)u1;
    nvv += (A)n1 * (A)v1;
  }
  if (a < a1) {
    const size_t j = (size_t)ci[a] * r + k;
    mu += (A)mv[a] * (A)U[j];
    nvv += (A)nv[a] * (A)V[j];
  }
}

// Row sums of VPT adjacent test vectors at once: acc[v] = sum over row
// [a0, a1) of val[a] X[ci[a] r + k0 + v], each in index order and in A as
// row_dot forms it; the VPT entries of a gathered row come in one vector
// load.
template <class A, class T, int VPT>
__device__ __forceinline__ void row_dot_v(int a0, int a1, const int *__restrict__ ci,
                                          const T *__restrict__ val, const T *__restrict__ X,
                                          int r, int k0, A (&acc)[VPT]) {
  typedef T vec __attribute__((ext_vector_type(VPT)));
#pragma unroll
  for (int v = 0; v < VPT; ++v) acc[v] = 0;
  int a = a0;
  for (; a + 4 <= a1; a += 4) {
    int c[4];
    T w[4];
    vec x[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      c[j] = ci[a + j];
      w[j] = val[a + j];
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) x[j] = *reinterpret_cast<const vec *>(X + (size_t)c[j] * r + k0);
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < VPT; ++v) acc[v] += (A)w[j] * (A)x[j][v];
  }
  for (; a < a1; ++a) {
    const T w = val[a];
    const vec x = *reinterpret_cast<const vec *>(X + (size_t)ci[a] * r + k0);
#pragma unroll
    for (int v = 0; v < VPT; ++v) acc[v] += (A)w * (A)x[v];
  }
}

// The same for row_dot2's pair (mv . U, nv . V) on one row of M
template <class A, class T, int VPT>
__device__ __forceinline__ void row_dot2_v(int a0, int a1, const int *__restrict__ ci,
                                           const T *__restrict__ mv, const T *__restrict__ nv,
                                           const T *__restrict__ U, const T *__restrict__ V,
                                           int r, int k0, A (&mu)[VPT], A (&nvv)[VPT]) {
  typedef T vec __attribute__((ext_vector_type(VPT)));
#pragma unroll
  for (int v = 0; v < VPT; ++v) mu[v] = nvv[v] = 0;
  for (int a = a0; a < a1; ++a) {
    const size_t j = (size_t)ci[a] * r + k0;
    const T m = mv[a], w = nv[a];
    const vec u = *reinterpret_cast<const vec *>(U + j), x = *reinterpret_cast<const vec *>(V + j);
#pragma unroll
    for (int v = 0; v < VPT; ++v) {
      mu[v] += (A)m * (A)u[v];
      nvv[v] += (A)w * (A)x[v];
    }
  }
}

// One simultaneous weighted-Jacobi step on all test vectors (Algorithm 1):
//   v_k <- v_k + omega D^-1 (sigma_k M u_k - B v_k)
//   u_k <- u_k + omega D^-1 (sigma_k N v_k - B^T u_k)     (k >= 1)
// with the sigma terms dropped for the homogeneous first pass. Both
// right-hand sides use the old vectors. A thread takes VPT adjacent columns
// k0 .. k0 + VPT - 1 of one row (VPT divides r), so a row's entries are
// read by r / VPT threads instead of r and each gather brings VPT values;
// the sums are those of one thread per column. Blocks renumbered
// XCD-contiguous.
template <class T, int VPT>
__global__ void __launch_bounds__(256)
    k_relax_pairs(int n, int r, const int *__restrict__ brp, const int *__restrict__ bci,
                  const T *__restrict__ bv, const int *__restrict__ trp,
                  const int *__restrict__ tci, const T *__restrict__ tv,
                  const int *__restrict__ mrp, const int *__restrict__ mci,
                  const T *__restrict__ mv, const T *__restrict__ nv, int identity_mn,
                  const T *__restrict__ dinv, T omega, int with_rhs,
                  const double *__restrict__ sigma, const T *__restrict__ U,
                  const T *__restrict__ V, T *__restrict__ Uo, T *__restrict__ Vo) {
  const long tid = (long)xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x;
  const int g = r / VPT;
  if (tid >= (long)n * g) return;
  const int i = (int)(tid / g), k0 = (int)(tid % g) * VPT;
  const size_t base = (size_t)i * r + k0;
  const T di = dinv[i];
  T bvk[VPT], btu[VPT];
  row_dot_v<T, T, VPT>(brp[i], brp[i + 1], bci, bv, V, r, k0, bvk);
  row_dot_v<T, T, VPT>(trp[i], trp[i + 1], tci, tv, U, r, k0, btu);
  T mu[VPT], nvv[VPT];
  if (with_rhs) {
    if (identity_mn) {
#pragma unroll
      for (int v = 0; v < VPT; ++v) {
        mu[v] = U[base + v];
        nvv[v] = V[base + v];
      }
    } else {
      row_dot2_v<T, T, VPT>(mrp[i], mrp[i + 1], mci, mv, nv, U, V, r, k0, mu, nvv);
    }
  }
#pragma unroll
  for (int v = 0; v < VPT; ++v) {
    const int k = k0 + v;
    T rhs_v = 0, rhs_u = 0;
    if (with_rhs) {
      const T sg = (T)sigma[k];
      rhs_v = sg * mu[v];
      rhs_u = sg * nvv[v];
    }
    const T uk = U[base + v], vk = V[base + v];
    Vo[base + v] = vk + omega * di * (rhs_v - bvk[v]);
    Uo[base + v] = k == 0 ? uk : uk + omega * di * (rhs_u - btu[v]);
  }
}

template <class T>
void relax_pairs(const Level &L, int r, T omega, int with_rhs, const double *sigma, const T *U,
                 const T *V, T *Uo, T *Vo, hipStream_t s) {
  // two columns per thread (tandem 2049^2 setup, all levels: 11.8 ms of
  // relaxation against 14.4 with one, 15.3 with four, 23.9 with eight)
  const int vpt = r % 2 == 0 ? 2 : 1;
  const long tot = (long)L.n * (r / vpt);
#define BAMG_RELAX(VPT)                                                                          \
  k_relax_pairs<T, VPT><<<ceil_div(tot, 256), 256, 0, s>>>(                                      \
      L.n, r, L.B.rp, L.B.ci, (const T *)L.Bv, L.Bt.rp, L.Bt.ci, (const T *)L.Btv, L.M.rp, L.M.ci, \
      (const T *)L.Mv, (const T *)L.Nv, L.identity_mn ? 1 : 0, (const T *)L.dinv, omega, with_rhs, \
      sigma, U, V, Uo, Vo)
  if (vpt == 2)
    BAMG_RELAX(2);
  else
    BAMG_RELAX(1);
#undef BAMG_RELAX
  LAUNCHCHK();
}

// Per-block partial sums, FP64, deterministic order. For each column k:
//   q0 = u.B v, q1 = u.M u, q2 = v.N v, q3 = |B v|^2, q4 = |B^T u|^2
// `which` bit 0: q0..q2, bit 1: q3, q4. A group of G lanes holds the
// columns of one row, VPT adjacent columns per lane (two where r is even,
// as in the relaxation); a block of 256 threads covers 256 / G rows per
// step. Partial t of column k from block b goes to part[(16 t + k) * nblk +
// b], so the finalisation reads each output's partials contiguously.
constexpr int kPPThreads = 256, kPPLanes = 16;

template <class T, int G, int VPT>
__global__ void __launch_bounds__(kPPThreads)
    k_pair_products(int n, int r, const int *__restrict__ brp, const int *__restrict__ bci,
                    const T *__restrict__ bv, const int *__restrict__ trp,
                    const int *__restrict__ tci, const T *__restrict__ tv,
                    const int *__restrict__ mrp, const int *__restrict__ mci,
                    const T *__restrict__ mv, const T *__restrict__ nv, int identity_mn,
                    const T *__restrict__ U, const T *__restrict__ V, int which,
                    double *__restrict__ part) {
  constexpr int kRows = kPPThreads / G, NC = G * VPT;
  __shared__ double sh[kPPThreads / kWave][5][NC];
  const int nblk = gridDim.x, vb = xcd_block(blockIdx.x, nblk);
  const int k0 = (threadIdx.x % G) * VPT;
  const int rowoff = threadIdx.x / G;
  double q[5][VPT];
#pragma unroll
  for (int t = 0; t < 5; ++t)
#pragma unroll
    for (int v = 0; v < VPT; ++v) q[t][v] = 0.0;
  if (k0 < r) {
    for (long i = (long)vb * kRows + rowoff; i < n; i += (long)nblk * kRows) {
      const size_t ik = (size_t)i * r + k0;
      double u[VPT], v[VPT], b[VPT];
#pragma unroll
      for (int c = 0; c < VPT; ++c) {
        u[c] = (double)U[ik + c];
        v[c] = (double)V[ik + c];
      }
      row_dot_v<double, T, VPT>(brp[i], brp[i + 1], bci, bv, V, r, k0, b);
      if (which & 1) {
        double mu[VPT], nvv[VPT];
        if (identity_mn) {
#pragma unroll
          for (int c = 0; c < VPT; ++c) {
            mu[c] = u[c];
            nvv[c] = v[c];
          }
        } else {
          row_dot2_v<double, T, VPT>(mrp[i], mrp[i + 1], mci, mv, nv, U, V, r, k0, mu, nvv);
        }
#pragma unroll
        for (int c = 0; c < VPT; ++c) {
          q[0][c] += u[c] * b[c];
          q[1][c] += u[c] * mu[c];
          q[2][c] += v[c] * nvv[c];
        }
      }
      if (which & 2) {
        double bt[VPT];
        row_dot_v<double, T, VPT>(trp[i], trp[i + 1], tci, tv, U, r, k0, bt);
#pragma unroll
        for (int c = 0; c < VPT; ++c) {
          q[3][c] += b[c] * b[c];
          q[4][c] += bt[c] * bt[c];
        }
      }
    }
  }
  // lanes l, l ^ G, l ^ 2G, ... of a wave share the columns k0 .. k0 + VPT - 1
#pragma unroll
  for (int t = 0; t < 5; ++t)
#pragma unroll
    for (int c = 0; c < VPT; ++c) {
      double x = q[t][c];
#pragma unroll
      for (int off = G; off < kWave; off <<= 1) x += __shfl_xor(x, off, kWave);
      q[t][c] = x;
    }
  const int w = threadIdx.x / kWave, l = threadIdx.x % kWave;
  if (l < G)
    for (int t = 0; t < 5; ++t)
      for (int c = 0; c < VPT; ++c) sh[w][t][k0 + c] = q[t][c];
  __syncthreads();
  if (threadIdx.x < 5 * NC) {
    const int t = threadIdx.x / NC, kk = threadIdx.x % NC;
    if (kk < r && ((t < 3) ? (which & 1) : (which & 2))) {
      double s = 0.0;
      for (int ww = 0; ww < kPPThreads / kWave; ++ww) s += sh[ww][t][kk];
      part[(size_t)(t * kPPLanes + kk) * nblk + vb] = s;
    }
  }
}

// lanes per row of the products: two columns each for even r (4 lanes up to
// r = 8, else 8), one each for odd r (8 lanes up to r = 8, else 16)
static int product_lanes(int r) { return r % 2 == 0 ? (r <= 8 ? 4 : 8) : (r <= 8 ? 8 : 16); }

// Blocks for the products on a level of n rows: one row per thread group
// while that fits in nmax blocks.
int product_blocks(int n, int r, int nmax) {
  const int rows = kPPThreads / product_lanes(r);
  return std::max(1, std::min(nmax, ceil_div(n, rows)));
}

template <class T>
int pair_products(const Level &L, int r, const T *U, const T *V, int which, double *part,
                  int nmax, hipStream_t s) {
  if (r > kPPLanes) fail(BAMG_E_ARG, "r above 16");
  const int nblk = product_blocks(L.n, r, nmax);
  const int g = product_lanes(r);
#define BAMG_PP(G, VPT)                                                                        \
  k_pair_products<T, G, VPT><<<nblk, kPPThreads, 0, s>>>(                                      \
      L.n, r, L.B.rp, L.B.ci, (const T *)L.Bv, L.Bt.rp, L.Bt.ci, (const T *)L.Btv, L.M.rp,    \
      L.M.ci, (const T *)L.Mv, (const T *)L.Nv, L.identity_mn ? 1 : 0, U, V, which, part)
  if (r % 2 == 0) {
    if (g == 4)
      BAMG_PP(4, 2);
    else
      BAMG_PP(8, 2);
  } else {
    if (g == 8)
      BAMG_PP(8, 1);
    else
      BAMG_PP(16, 1);
  }
#undef BAMG_PP
  LAUNCHCHK();
  return nblk;
}

// out[16 t + k] = sum over the nblk partials, block k per column, fixed
// reduction tree; then, in the same block, the column's scalar that the
// products feed (epi 1: sigma_k, Algorithm 1; epi 2: the normalisation
// scales of v_k and u_k).
__global__ void __launch_bounds__(256)
    k_finalize_products(const double *__restrict__ part, int nblk, int which, int epi,
                        double *__restrict__ out, double *__restrict__ aux) {
  __shared__ double sh[4];
  const int k = blockIdx.x;
  double q[5] = {0, 0, 0, 0, 0};
  for (int t = 0; t < 5; ++t) {
    if (!((t < 3) ? (which & 1) : (which & 2))) continue;
    const double *p = part + (size_t)(t * kPPLanes + k) * nblk;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblk; b += 256) s += p[b];
    q[t] = block_sum<256>(s, sh);
    if (threadIdx.x == 0) out[t * kPPLanes + k] = q[t];
  }
  if (threadIdx.x != 0) return;
  if (epi == 1) {
    const double den = sqrt(q[1] * q[2]);
    aux[k] = den > 0.0 ? q[0] / den : 0.0;
  } else if (epi == 2) {
    aux[k] = q[2] > 0.0 ? 1.0 / sqrt(q[2]) : 1.0;
    aux[kPPLanes + k] = (k > 0 && q[1] > 0.0) ? 1.0 / sqrt(q[1]) : 1.0;
  }
}

void finalize_products(const double *part, int nblk, int r, int which, int epi, double *out,
                       double *aux, hipStream_t s) {
  k_finalize_products<<<r, 256, 0, s>>>(part, nblk, which, epi, out, aux);
  LAUNCHCHK();
}

// omega_k = 1/||B v_k||^2 divided by the largest; same for u_k with B^T, k >= 1
__global__ void k_ls_weights(const double *__restrict__ q, int r, double *__restrict__ wv,
                             double *__restrict__ wu) {
  if (threadIdx.x != 0) return;
  const double tiny = 2.2250738585072014e-308;
  double minv = INFINITY, minu = INFINITY;
  double a[kPPLanes], b[kPPLanes];
  for (int k = 0; k < r; ++k) {
    a[k] = fmax(q[3 * kPPLanes + k], tiny);
    minv = fmin(minv, a[k]);
    b[k] = fmax(q[4 * kPPLanes + k], tiny);
    if (k > 0) minu = fmin(minu, b[k]);
  }
  for (int k = 0; k < r; ++k) {
    wv[k] = minv / a[k];
    wu[k] = k > 0 ? minu / b[k] : 0.0;
  }
}
void ls_weights(const double *prod, int r, double *wv, double *wu, hipStream_t s) {
  k_ls_weights<<<1, 64, 0, s>>>(prod, r, wv, wu);
  LAUNCHCHK();
}

template <class T>
__global__ void k_scale_columns(T *__restrict__ X, int n, int r, const double *__restrict__ sc,
                                int skip0) {
  long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long)n * r) return;
  const int k = (int)(idx % r);
  if (skip0 && k == 0) return;
  X[idx] = (T)((double)X[idx] * sc[k]);
}
template <class T>
void scale_columns(T *X, int n, int r, const double *scale, int skip0, hipStream_t s) {
  long tot = (long)n * r;
  if (!tot) return;
  k_scale_columns<T><<<ceil_div(tot, 256), 256, 0, s>>>(X, n, r, scale, skip0);
  LAUNCHCHK();
}

// ============================================================ Kaczmarz colouring
// Greedy distance-2 colouring of the rows in decreasing priority (key, i),
// key the first Philox word of counter (i, 0, 3, 0), key (0x4b41435a, 0):
// rows sharing a column get different colours. Computed in rounds: a row
// whose conflicting uncoloured rows all have lower priority takes the
// smallest colour unused by its coloured conflicts; this reproduces the
// sequential greedy order.
__global__ void k_col_keys(int n, uint64_t *__restrict__ key, int *__restrict__ colour) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  key[i] = philox_word0((uint64_t)i, 0, 3, 0, 0x4b41435aULL, 0);
  colour[i] = -1;
}

__global__ void k_col_round(int n, const int *__restrict__ rp, const int *__restrict__ ci,
                            const int *__restrict__ crp, const int *__restrict__ cci,
                            const uint64_t *__restrict__ key, const int *__restrict__ colour_in,
                            int *__restrict__ colour_out, int *__restrict__ remaining) {
  int v = blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  if (colour_in[v] >= 0) {
    colour_out[v] = colour_in[v];
    return;
  }
  const uint64_t kv = key[v];
  uint64_t used_lo = 0, used_hi = 0;  // colours 0..127
  for (int a = rp[v]; a < rp[v + 1]; ++a) {
    const int j = ci[a];
    for (int b = crp[j]; b < crp[j + 1]; ++b) {
      const int w = cci[b];
      if (w == v) continue;
      const int cw = colour_in[w];
      if (cw < 0) {
        const uint64_t kw = key[w];
        if (kw > kv || (kw == kv && w > v)) {
          colour_out[v] = -1;
          atomicAdd(remaining, 1);
          return;
        }
      } else if (cw < 64) {
        used_lo |= 1ull << cw;
      } else if (cw < 128) {
        used_hi |= 1ull << (cw - 64);
      }
    }
  }
  int c = 0;
  if (~used_lo)
    c = __ffsll((long long)~used_lo) - 1;
  else if (~used_hi)
    c = 64 + __ffsll((long long)~used_hi) - 1;
  else
    c = 128;
  colour_out[v] = c;
}

__global__ void k_count_colour(const int *__restrict__ colour, int n, int *__restrict__ cnt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) atomicAdd(&cnt[colour[i]], 1);
}

__global__ void k_order_by_colour(const int *__restrict__ colour, int n,
                                  const int *__restrict__ off, int *__restrict__ order) {
  // stable: thread-per-colour scan over rows keeps rows ascending within a colour
  int c = blockIdx.x * blockDim.x + threadIdx.x;
  int p = off[c];
  for (int i = 0; i < n; ++i)
    if (colour[i] == c) order[p++] = i;
}

void row_colouring(Pool &pool, const Csr &A, const Csr &At, int *colour, int &ncol, int *&order,
                   std::vector<int> &offsets, hipStream_t s) {
  const int n = A.nr;
  uint64_t *key = pool.get<uint64_t>(n);
  int *tmp = pool.get<int>(n);
  int *rem = pool.get<int>(1);
  k_col_keys<<<ceil_div(n, 256), 256, 0, s>>>(n, key, colour);
  LAUNCHCHK();
  int *cin = colour, *cout = tmp;
  for (int round = 0;; ++round) {
    if (round > n + 1) fail(BAMG_E_DEVICE, "colouring did not terminate");
    fill_i32(rem, 0, 1, s);
    k_col_round<<<ceil_div(n, 256), 256, 0, s>>>(n, A.rp, A.ci, At.rp, At.ci, key, cin, cout, rem);
    LAUNCHCHK();
    std::swap(cin, cout);
    if (read_int(rem, s) == 0) break;
  }
  if (cin != colour)
    HIPCHK(hipMemcpyAsync(colour, cin, sizeof(int) * n, hipMemcpyDeviceToDevice, s));
  // number of colours
  int *cnt = pool.get<int>(130);
  fill_i32(cnt, 0, 130, s);
  k_count_colour<<<ceil_div(n, 256), 256, 0, s>>>(colour, n, cnt);
  LAUNCHCHK();
  std::vector<int> hc(130);
  HIPCHK(hipMemcpyAsync(hc.data(), cnt, sizeof(int) * 130, hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (hc[128] || hc[129]) fail(BAMG_E_ARG, "more than 128 colours in the Kaczmarz colouring");
  ncol = 0;
  for (int c = 0; c < 128; ++c)
    if (hc[c]) ncol = c + 1;
  offsets.assign(ncol + 1, 0);
  for (int c = 0; c < ncol; ++c) offsets[c + 1] = offsets[c] + hc[c];
  int *doff = pool.get<int>(ncol + 1);
  HIPCHK(hipMemcpyAsync(doff, offsets.data(), sizeof(int) * (ncol + 1), hipMemcpyHostToDevice, s));
  order = pool.get<int>(n);
  k_order_by_colour<<<1, ncol, 0, s>>>(colour, n, doff, order);
  LAUNCHCHK();
  HIPCHK(hipStreamSynchronize(s));
  pool.release(key);
  pool.release(tmp);
  pool.release(rem);
  pool.release(cnt);
  pool.release(doff);
}

template <class T>
__global__ void k_row_inv_norms(int n, const int *__restrict__ rp, const T *__restrict__ v,
                                T *__restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int a = rp[i]; a < rp[i + 1]; ++a) s += (double)v[a] * (double)v[a];
  out[i] = (T)(s > 0.0 ? 1.0 / s : 0.0);
}
template <class T>
void row_inv_norms(const Csr &A, const T *val, T *out, hipStream_t s) {
  if (!out || !val) fail(BAMG_E_DEVICE, "row_inv_norms: missing buffer");
  k_row_inv_norms<T><<<ceil_div(A.nr, 256), 256, 0, s>>>(A.nr, A.rp, val, out);
  LAUNCHCHK();
}

#define INST(T)                                                                              \
  template void spgemm_numeric<T>(const Csr &, const T *, const Csr &, const T *, const Csr &, \
                                  T *, int *, hipStream_t);                                  \
  template void fill_transfer_identity<T>(const Level &, T *, T *, hipStream_t);             \
  template void ls_fit<T>(const Level &, int, int, const T *, const T *, const double *,      \
                          const double *, int, int, T *, T *, hipStream_t);                  \
  template void dinv_from_diag<T>(const Level &, const T *, T *, int *, bool, hipStream_t);               \
  template void inject<T>(const int *, int, int, const T *, T *, hipStream_t);               \
  template void spmm<T>(const Csr &, const T *, int, const T *, T *, int, hipStream_t);      \
  template void relax_pairs<T>(const Level &, int, T, int, const double *, const T *,        \
                               const T *, T *, T *, hipStream_t);                            \
  template int pair_products<T>(const Level &, int, const T *, const T *, int, double *,    \
                                 int, hipStream_t);                                          \
  template void scale_columns<T>(T *, int, int, const double *, int, hipStream_t);           \
  template void row_inv_norms<T>(const Csr &, const T *, T *, hipStream_t);
INST(double)
INST(float)
#undef INST

}  // namespace bamg
