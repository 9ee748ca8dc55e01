// 6-connected components of every isoband (Sec. 3.1), numbered by (band,
// smallest linear index) -- the hierarchical order of Sec. 3.2.4 / Fig. 5.
//
// Pipeline (all labels are linear voxel indices until the final relabel):
//  1. brick-local union-find in LDS over 32x8x8 bricks; roots are the
//     smallest local index, which is also the smallest global index because
//     the local and global raster orders agree;
//  2. union across the three low faces of every brick in global memory
//     (lock-free union by smaller root, so a root is always the smallest
//     index of its component); a face pair whose predecessor along the face
//     already links the same two components is skipped;
//  3. roots (label[v] == v) are compacted in linear order, then stably sorted
//     by band: the position is the canonical component id;
//  4. every voxel finds its root and takes the root's id; component sizes
//     are summed per tile in an LDS hash table, then one atomic per distinct
//     component and tile.
#include "common.h"

namespace lsrvt {

namespace {

constexpr int CX = 32, CY = 8, CZ = 8;
constexpr int kBrick = CX * CY * CZ;  // 2048 voxels
constexpr int kCCThreads = 256;
constexpr uint8_t kOutside = 255;  // band marker for voxels beyond the volume

struct BrickGrid {
  int32_t nbx, nby, nbz;
};

__device__ __forceinline__ uint32_t ld_relaxed(uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t lds_relaxed(uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ uint32_t find_lds(uint32_t *p, uint32_t x) {
  uint32_t q = lds_relaxed(&p[x]);
  while (q != x) {
    x = q;
    q = lds_relaxed(&p[x]);
  }
  return x;
}

// Lock-free union: link the larger root below the smaller one.  p[x] <= x
// always holds, so no cycle can form; a failed link (the root was linked
// concurrently) continues with the value the atomic returned.
__device__ void unite_lds(uint32_t *p, uint32_t a, uint32_t b) {
  while (true) {
    a = find_lds(p, a);
    b = find_lds(p, b);
    if (a == b) return;
    if (a < b) {
      uint32_t t = a;
      a = b;
      b = t;
    }
    uint32_t old = atomicMin(&p[a], b);
    if (old == a) return;
    a = old;
  }
}

__device__ uint32_t find_global(uint32_t *p, uint32_t x) {
  uint32_t q = ld_relaxed(&p[x]);
  while (q != x) {
    x = q;
    q = ld_relaxed(&p[x]);
  }
  return x;
}

__device__ void unite_global(uint32_t *p, uint32_t a, uint32_t b) {
  while (true) {
    a = find_global(p, a);
    b = find_global(p, b);
    if (a == b) return;
    if (a < b) {
      uint32_t t = a;
      a = b;
      b = t;
    }
    uint32_t old = atomicMin(&p[a], b);
    if (old == a) return;
    a = old;
  }
}

__global__ __launch_bounds__(kCCThreads) void k_cc_local(const uint8_t *__restrict__ band, Geom g, BrickGrid bg,
                                                         uint32_t *__restrict__ label) {
  __shared__ uint8_t sb[kBrick];
  __shared__ uint32_t sp[kBrick];
  const int b = blockIdx.x;
  const int bx = b % bg.nbx, by = (b / bg.nbx) % bg.nby, bz = b / (bg.nbx * bg.nby);
  const int x0 = bx * CX, y0 = by * CY, z0 = bz * CZ;
  bool mixed = false;  // the brick holds more than one band (or voxels beyond the volume)
  uint8_t first = 0;
  for (int li = threadIdx.x; li < kBrick; li += kCCThreads) {
    int lx = li % CX, ly = (li / CX) % CY, lz = li / (CX * CY);
    int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
    bool valid = gx < g.nx && gy < g.ny && gz < g.nz;
    const uint8_t bv = valid ? band[gx + (int64_t)g.nx * (gy + (int64_t)g.ny * gz)] : kOutside;
    sb[li] = bv;
    if (li == (int)threadIdx.x) first = bv;
    mixed |= bv != first || bv == kOutside;
  }
  __syncthreads();
  // one band over the whole brick: every voxel's root is the brick's first voxel
  mixed |= first != sb[0];
  if (!__syncthreads_or(mixed)) {
    const int64_t gr = x0 + (int64_t)g.nx * (y0 + (int64_t)g.ny * z0);
    for (int li = threadIdx.x; li < kBrick; li += kCCThreads) {
      int lx = li % CX, ly = (li / CX) % CY, lz = li / (CX * CY);
      label[(x0 + lx) + (int64_t)g.nx * ((y0 + ly) + (int64_t)g.ny * (z0 + lz))] = (uint32_t)gr;
    }
    return;
  }
  // every voxel starts linked to the first voxel of its run of equal band
  // along x (a valid forest: parents never exceed their children), so only
  // the y and z neighbours need unions
  for (int li = threadIdx.x; li < kBrick; li += kCCThreads) {
    const uint8_t bv = sb[li];
    int st = li;
    while ((st % CX) > 0 && sb[st - 1] == bv) --st;
    sp[li] = (uint32_t)st;
  }
  __syncthreads();
  for (int li = threadIdx.x; li < kBrick; li += kCCThreads) {
    uint8_t bv = sb[li];
    if (bv == kOutside) continue;
    int ly = (li / CX) % CY, lz = li / (CX * CY);
    if (ly > 0 && sb[li - CX] == bv) unite_lds(sp, li, li - CX);
    if (lz > 0 && sb[li - CX * CY] == bv) unite_lds(sp, li, li - CX * CY);
  }
  __syncthreads();
  for (int li = threadIdx.x; li < kBrick; li += kCCThreads) {
    if (sb[li] == kOutside) continue;
    uint32_t r = find_lds(sp, li);
    int lx = li % CX, ly = (li / CX) % CY, lz = li / (CX * CY);
    int rx = r % CX, ry = (r / CX) % CY, rz = r / (CX * CY);
    int64_t gi = (x0 + lx) + (int64_t)g.nx * ((y0 + ly) + (int64_t)g.ny * (z0 + lz));
    int64_t gr = (x0 + rx) + (int64_t)g.nx * ((y0 + ry) + (int64_t)g.ny * (z0 + rz));
    label[gi] = (uint32_t)gr;
  }
}

// Union across the low x, y and z faces of each brick.
__global__ __launch_bounds__(kCCThreads) void k_cc_merge(const uint8_t *__restrict__ band, Geom g, BrickGrid bg,
                                                         uint32_t *label) {
  const int b = blockIdx.x;
  const int bx = b % bg.nbx, by = (b / bg.nbx) % bg.nby, bz = b / (bg.nbx * bg.nby);
  const int x0 = bx * CX, y0 = by * CY, z0 = bz * CZ;
  const int64_t sx = 1, sy = g.nx, sz = (int64_t)g.nx * g.ny;
  constexpr int nfx = CY * CZ, nfy = CX * CZ, nfz = CX * CY;
  for (int t = threadIdx.x; t < nfx + nfy + nfz; t += kCCThreads) {
    int lx, ly, lz;
    int64_t across, prev;  // offset to the neighbour across the face; to the predecessor along the face
    bool has_prev;
    if (t < nfx) {  // -x face: (0, ly, lz), predecessor along y
      if (x0 == 0) continue;
      lx = 0;
      ly = t % CY;
      lz = t / CY;
      across = sx;
      prev = sy;
      has_prev = ly > 0;
    } else if (t < nfx + nfy) {  // -y face: (lx, 0, lz), predecessor along x
      if (y0 == 0) continue;
      int u = t - nfx;
      lx = u % CX;
      ly = 0;
      lz = u / CX;
      across = sy;
      prev = sx;
      has_prev = lx > 0;
    } else {  // -z face: (lx, ly, 0), predecessor along x
      if (z0 == 0) continue;
      int u = t - nfx - nfy;
      lx = u % CX;
      ly = u / CX;
      lz = 0;
      across = sz;
      prev = sx;
      has_prev = lx > 0;
    }
    int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
    if (gx >= g.nx || gy >= g.ny || gz >= g.nz) continue;
    int64_t v = gx + sy * gy + sz * gz;
    int64_t w = v - across;
    uint8_t bv = band[v];
    if (band[w] != bv) continue;
    if (has_prev && band[v - prev] == bv && band[w - prev] == bv) continue;  // implied by the predecessor pair
    unite_global(label, label[v], label[w]);
  }
}

constexpr int kTile = 4096;  // voxels per root-compaction tile (256 threads x 16)

__global__ __launch_bounds__(256) void k_root_count(const uint32_t *__restrict__ label, int64_t n,
                                                    uint32_t *__restrict__ tile_count) {
  __shared__ uint32_t wsum[4];
  int64_t base = (int64_t)blockIdx.x * kTile;
  uint32_t c = 0;
  for (int i = threadIdx.x; i < kTile; i += 256) {
    int64_t v = base + i;
    if (v < n && label[v] == (uint32_t)v) ++c;
  }
  c = wave_sum_u32(c);
  if (lane_id() == 0) wsum[threadIdx.x / kWave] = c;
  __syncthreads();
  if (threadIdx.x == 0) tile_count[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// Write the roots of each tile in increasing linear order, plus their bands.
__global__ __launch_bounds__(256) void k_root_scatter(const uint32_t *__restrict__ label, const uint8_t *__restrict__ band,
                                                      int64_t n, const uint32_t *__restrict__ tile_off,
                                                      uint32_t *__restrict__ roots, uint8_t *__restrict__ root_band) {
  __shared__ uint32_t wcnt[4];
  __shared__ uint32_t base_s;
  if (threadIdx.x == 0) base_s = tile_off[blockIdx.x];
  __syncthreads();
  int64_t base = (int64_t)blockIdx.x * kTile;
  const int wid = threadIdx.x / kWave;
  for (int i0 = 0; i0 < kTile; i0 += 256) {
    int64_t v = base + i0 + threadIdx.x;
    bool is_root = v < n && label[v] == (uint32_t)v;
    uint64_t m = __ballot(is_root);
    if (lane_id() == 0) wcnt[wid] = (uint32_t)__popcll(m);
    __syncthreads();
    uint32_t off = base_s;
    for (int w = 0; w < wid; ++w) off += wcnt[w];
    if (is_root) {
      uint32_t pos = off + (uint32_t)__popcll(m & lanemask_lt());
      roots[pos] = (uint32_t)v;
      root_band[pos] = band[v];
    }
    __syncthreads();
    if (threadIdx.x == 0) base_s += wcnt[0] + wcnt[1] + wcnt[2] + wcnt[3];
    __syncthreads();
  }
}

__global__ void k_cc_tables(const uint32_t *__restrict__ roots, const uint8_t *__restrict__ root_band,
                            const uint32_t *__restrict__ pos, uint32_t n_comp, int write_tables,
                            uint32_t *__restrict__ comp, uint8_t *__restrict__ comp_band,
                            uint32_t *__restrict__ comp_first, uint64_t *__restrict__ comp_size) {
  uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_comp) return;
  uint32_t r = roots[i], c = pos[i];
  comp[r] = c;  // the root voxel carries its component id for the relabel pass
  if (write_tables) {
    comp_band[c] = root_band[i];
    comp_first[c] = r;
    comp_size[c] = 0;
  }
}

// Relabel: one workgroup per 64x8x8 tile, each thread walks 16 consecutive
// voxels of a row; the root of a label is cached across a run of equal labels;
// component sizes accumulate per run in an LDS hash table and are flushed with
// one atomic per distinct component in the tile.
constexpr int RX = 64, RY = 8, RZ = 8;
constexpr int kRelCap = 512;

__global__ __launch_bounds__(256) void k_cc_relabel(const uint32_t *__restrict__ label, Geom g, uint32_t *comp,
                                                    uint64_t *comp_size, int count_sizes) {
  __shared__ uint32_t tkey[kRelCap], tcnt[kRelCap];
  const int t = threadIdx.x;
  const int ntx = (g.nx + RX - 1) / RX, nty = (g.ny + RY - 1) / RY, ntz = (g.nz + RZ - 1) / RZ;
  const int64_t ntiles = (int64_t)ntx * nty * ntz;
  for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    for (int i = t; i < kRelCap; i += 256) {
      tkey[i] = kNone;
      tcnt[i] = 0;
    }
    __syncthreads();
    const int ttx = (int)(tile % ntx), tty = (int)((tile / ntx) % nty), ttz = (int)(tile / ((int64_t)ntx * nty));
    const int x0 = ttx * RX + (t & 3) * 16, y = tty * RY + ((t >> 2) & 7), z = ttz * RZ + (t >> 5);
    if (y < g.ny && z < g.nz && x0 < g.nx) {
      const int64_t base = (int64_t)g.nx * (y + (int64_t)g.ny * z);
      const int xe = x0 + 16 < g.nx ? x0 + 16 : g.nx;
      uint32_t last_lab = kNone, last_cid = kNone, run_cid = kNone, run_n = 0;
      auto flush = [&]() {
        if (run_n && count_sizes) {
          int sl = lds_slot<kRelCap>(tkey, run_cid);
          if (sl >= 0)
            atomicAdd(&tcnt[sl], run_n);
          else
            atomicAdd((unsigned long long *)&comp_size[run_cid], (unsigned long long)run_n);
        }
      };
      for (int x = x0; x < xe; ++x) {
        const int64_t v = base + x;
        const uint32_t lab = label[v];
        uint32_t r = lab;
        uint32_t cid;
        if (r == last_lab) {
          cid = last_cid;
        } else {
          last_lab = r;
          uint32_t q = label[r];
          while (q != r) {
            r = q;
            q = label[r];
          }
          cid = comp[r];
          last_cid = cid;
        }
        if (lab != (uint32_t)v) comp[v] = cid;
        if (cid != run_cid) {
          flush();
          run_cid = cid;
          run_n = 0;
        }
        ++run_n;
      }
      flush();
    }
    __syncthreads();
    if (count_sizes)
      for (int i = t; i < kRelCap; i += 256)
        if (tkey[i] != kNone) atomicAdd((unsigned long long *)&comp_size[tkey[i]], (unsigned long long)tcnt[i]);
    __syncthreads();
  }
}

struct CCLayout {
  uint32_t *label, *tile_count, *tile_off, *roots, *pos, *bucket;
  uint8_t *root_band;
  void *sort_work;
  size_t sort_bytes;
  void *scan_work;
  size_t scan_bytes;
};

template <class A>
void cc_layout(A &a, int64_t n, CCLayout *L) {
  int64_t ntiles = (n + kTile - 1) / kTile;
  auto t0 = a.template take<uint32_t>(n);
  auto t1 = a.template take<uint32_t>(ntiles);
  auto t2 = a.template take<uint32_t>(ntiles + 1);
  auto t3 = a.template take<uint32_t>(n);
  auto t4 = a.template take<uint32_t>(n);
  auto t5 = a.template take<uint32_t>(257);
  auto t6 = a.template take<uint8_t>(n);
  if (L) {
    L->label = t0;
    L->tile_count = t1;
    L->tile_off = t2;
    L->roots = t3;
    L->pos = t4;
    L->bucket = t5;
    L->root_band = t6;
  }
}

}  // namespace

}  // namespace lsrvt

using namespace lsrvt;

namespace {
struct SizerT : Sizer {
  template <class T>
  T *take(size_t c) {
    Sizer::take<T>(c);
    return nullptr;
  }
};
}  // namespace

extern "C" size_t lsrvt_components_workspace(lsrvt_dims dims, int32_t n_bands) {
  (void)n_bands;
  Geom g;
  if (make_geom(dims, g)) return 0;
  SizerT z;
  cc_layout(z, g.n, (CCLayout *)nullptr);
  size_t sort_ws = StableSort8::workspace(g.n);
  size_t scan_ws = ScanU32::workspace((g.n + kTile - 1) / kTile);
  return z.off + (sort_ws > scan_ws ? sort_ws : scan_ws) + 256;
}

extern "C" int32_t lsrvt_components(const uint8_t *d_band, lsrvt_dims dims, int32_t n_bands, uint32_t *d_comp,
                                    uint32_t cap_comp, uint8_t *d_comp_band, uint64_t *d_comp_size,
                                    uint32_t *d_comp_first, uint32_t *d_band_offset, uint32_t *h_n_comp,
                                    void *d_work, size_t work_bytes, void *stream) {
  Geom g;
  int32_t st = make_geom(dims, g);
  if (st) return st;
  if (n_bands < 1 || n_bands > 255) return LSRVT_EINVAL;
  if (!d_band || !d_comp || !h_n_comp) return LSRVT_EINVAL;
  if (cap_comp > 0 && (!d_comp_band || !d_comp_size || !d_comp_first)) return LSRVT_EINVAL;
  if (!d_band_offset) return LSRVT_EINVAL;
  st = check_work(d_work, work_bytes, lsrvt_components_workspace(dims, n_bands));
  if (st) return st;
  hipStream_t s = as_stream(stream);

  Carve cv(d_work, work_bytes);
  CCLayout L;
  cc_layout(cv, g.n, &L);
  if (!cv.ok) return LSRVT_EWORKSPACE;
  void *rest = cv.base + cv.off;
  size_t rest_bytes = cv.size - cv.off;

  BrickGrid bg{(g.nx + CX - 1) / CX, (g.ny + CY - 1) / CY, (g.nz + CZ - 1) / CZ};
  unsigned nbricks = (unsigned)((int64_t)bg.nbx * bg.nby * bg.nbz);
  hipLaunchKernelGGL(k_cc_local, dim3(nbricks), dim3(kCCThreads), 0, s, d_band, g, bg, L.label);
  hipLaunchKernelGGL(k_cc_merge, dim3(nbricks), dim3(kCCThreads), 0, s, d_band, g, bg, L.label);
  int64_t ntiles = (g.n + kTile - 1) / kTile;
  hipLaunchKernelGGL(k_root_count, dim3((unsigned)ntiles), dim3(256), 0, s, L.label, g.n, L.tile_count);
  LSRVT_LAUNCHED();
  st = ScanU32::run(L.tile_count, ntiles, L.tile_off, rest, rest_bytes, s);
  if (st) return st;
  hipLaunchKernelGGL(k_root_scatter, dim3((unsigned)ntiles), dim3(256), 0, s, L.label, d_band, g.n, L.tile_off,
                     L.roots, L.root_band);
  LSRVT_LAUNCHED();
  uint32_t n_comp = 0;
  {
    const int32_t rc_ = read_words(L.tile_off + ntiles, 1, &n_comp, s);
    if (rc_) return rc_;
  }
  *h_n_comp = n_comp;
  st = StableSort8::run(L.root_band, n_comp, L.pos, L.bucket, rest, rest_bytes, s);
  if (st) return st;
  const int write_tables = n_comp <= cap_comp;
  if (n_comp > 0) {
    hipLaunchKernelGGL(k_cc_tables, dim3((n_comp + 255) / 256), dim3(256), 0, s, L.roots, L.root_band, L.pos, n_comp,
                       write_tables, d_comp, d_comp_band, d_comp_first, d_comp_size);
    LSRVT_LAUNCHED();
  }
  {
    const int64_t nt = (int64_t)((g.nx + RX - 1) / RX) * ((g.ny + RY - 1) / RY) * ((g.nz + RZ - 1) / RZ);
    hipLaunchKernelGGL(k_cc_relabel, dim3((unsigned)(nt < 65535 ? nt : 65535)), dim3(256), 0, s, L.label, g, d_comp,
                       d_comp_size, write_tables);
  }
  LSRVT_LAUNCHED();
  if (!write_tables) return LSRVT_ECAPACITY;
  LSRVT_HIP(hipMemcpyAsync(d_band_offset, L.bucket, sizeof(uint32_t) * (n_bands + 1), hipMemcpyDeviceToDevice, s));
  return LSRVT_OK;
}
