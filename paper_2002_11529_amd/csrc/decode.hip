// UT raw-bank decoding (Section IV of the paper) for gfx950.
//
// One wavefront handles one unit = (event, layer) = S consecutive banks whose words are contiguous.
//   k_decode_count: per unit, bank-offset checks and the number of valid words (one read of the
//     words);
//   k_decode_scan: one workgroup scans the unit sums into the first hit of every unit;
//   k_decode: per unit, words staged in LDS, stable compaction of the valid words (ballot + mbcnt),
//     local hit offsets of the banks, sort inside each bank by word value (a counting sort of the
//     chunk's hits on per-bank word bins, then a rank inside each bin), decode and coalesced store
//     of the six hit fields.
// The paper's seven kernels (count, three-kernel prefix sum, pre-decode, find permutation, decode
// in order; Table "Kernel configuration for UT decoding") become these two; the order inside a bank
// is by x (the word value) rather than by y.
#include <mutex>

#include "decode_unit.hpp"

namespace utc {

constexpr int kScanTmp = 17;   // block_exclusive_scan scratch (<= 1024 threads)

__global__ void __launch_bounds__(1024)
k_decode_count(Geom g, const uint16_t* __restrict__ words, const uint32_t* __restrict__ bank_offsets,
               int n_units, uint32_t* __restrict__ unit_sum, uint32_t* flags)
{
  extern __shared__ __align__(16) uint32_t s_off_all[];
  const int wid = threadIdx.x / kWave, nwaves = blockDim.x / kWave;
  WaveScratch ws{};
  ws.off = s_off_all + (size_t)wid * (g.S + 1);
  for (int u = blockIdx.x * nwaves + wid; u < n_units; u += gridDim.x * nwaves) {
    const UnitCount st = unit_count(g, words, bank_offsets, (int64_t)u * g.S, ws, flags);
    if (lane_id() == 0) unit_sum[u] = st.T;
    wave_sync();
  }
}

// One workgroup: exclusive scan of the unit sums into the first hit of every unit.  Each wave scans
// kScanRows consecutive rows of 64 values (coalesced loads, a DPP scan per row carried along the
// rows), the wave totals are scanned across the workgroup, and passes of 64 * kScanRows * waves
// values follow each other.
constexpr int kScanRows = 16;

__global__ void __launch_bounds__(1024)
k_decode_scan(const uint32_t* __restrict__ unit_sum, int n_units, uint32_t* __restrict__ unit_base,
              uint32_t* __restrict__ hit_offsets_end)
{
  __shared__ uint32_t tmp[kScanTmp];
  const int lane = lane_id();
  const int wid = threadIdx.x / kWave, nw = blockDim.x / kWave;
  uint32_t carry = 0;   // all values of the previous passes
  for (int64_t base = 0; base < n_units; base += (int64_t)nw * kWave * kScanRows) {
    const int64_t seg = base + (int64_t)wid * kWave * kScanRows;
    uint32_t v[kScanRows], ex[kScanRows];
#pragma unroll
    for (int r = 0; r < kScanRows; ++r) {
      const int64_t i = seg + r * kWave + lane;
      v[r] = i < n_units ? unit_sum[i] : 0u;
    }
    uint32_t run = 0;   // this wave's values before row r
#pragma unroll
    for (int r = 0; r < kScanRows; ++r) {
      const uint32_t x = wave_inclusive_scan(v[r]);
      ex[r] = run + x - v[r];
      run += (uint32_t)__builtin_amdgcn_readlane((int)x, kWave - 1);
    }
    // the waves' totals (carried by their last lane) scanned across the workgroup
    uint32_t tot;
    const uint32_t woff = block_exclusive_scan(lane == kWave - 1 ? run : 0u, tmp, &tot);
#pragma unroll
    for (int r = 0; r < kScanRows; ++r) {
      const int64_t i = seg + r * kWave + lane;
      if (i < n_units) unit_base[i] = carry + woff + ex[r];
    }
    carry += tot;
  }
  if (threadIdx.x == 0) {
    unit_base[n_units] = carry;
    *hit_offsets_end = carry;
  }
}

__global__ void __launch_bounds__(1024)
k_decode(Geom g, const uint16_t* __restrict__ words, const uint32_t* __restrict__ bank_offsets,
         int n_units, int cap, int64_t capacity, const uint32_t* __restrict__ unit_base,
         uint32_t* __restrict__ hit_offsets, HitsOut out, uint32_t* flags)
{
  extern __shared__ __align__(16) char smem[];
  const int wid = threadIdx.x / kWave, nwaves = blockDim.x / kWave;
  const WaveScratch ws = carve_scratch(smem + (size_t)wid * wave_scratch_bytes(g.S, cap), g.S, cap);
  for (int u = blockIdx.x * nwaves + wid; u < n_units; u += gridDim.x * nwaves) {
    const int64_t b0 = (int64_t)u * g.S;
    const UnitCount st = unit_count(g, words, bank_offsets, b0, ws, flags, u % kLayers);
    unit_write(g, words, u % kLayers, b0, unit_base[u], st, ws, capacity, hit_offsets, out, flags);
    wave_sync();
  }
}

}  // namespace utc

using namespace utc;

extern "C" size_t ut_decode_workspace_bytes(int32_t n_events, int32_t n_sectors)
{
  (void)n_sectors;
  if (n_events < 0) return 0;
  const size_t units = (size_t)n_events * kLayers;
  return ((2 * units + 1) * sizeof(uint32_t) + 255) / 256 * 256;
}

// The three launches of a decode call; unit_sum holds 2 * n_events * 4 + 1 words of device memory
// (the unit sums, then the unit bases), whatever its content.
static utc_status decode_launch(const utc_geometry* geom, const uint16_t* words,
                                const uint32_t* bank_offsets, int32_t n_events, int64_t hit_capacity,
                                uint32_t* hit_offsets, uint32_t* lhcbid, float* z, float* u,
                                float* y_begin, float* y_end, float* weight, uint32_t* error_flags,
                                uint32_t* unit_sum, const utc_launch_config* launch,
                                hipStream_t stream)
{
  const int S = geom->n_sectors;
  const int n_units = n_events * kLayers;
  uint32_t* unit_base = unit_sum + n_units;
  const Geom g = make_geom(*geom);
  const size_t tile = (launch && launch->window_tile > 0) ? (size_t)launch->window_tile * 1024
                                                          : kWaveLdsDefault;
  const int cap = chunk_words(S, tile);
  int block = launch ? launch->block : 256;
  while (!launch && block > kWave && (size_t)(block / kWave) * wave_scratch_bytes(S, cap) > 160 * 1024)
    block -= kWave;
  const int waves = block / kWave;
  const size_t lds = (size_t)waves * wave_scratch_bytes(S, cap);
  if (lds > 160 * 1024) return UTC_ERR_ARG;
  (void)hipGetLastError();  // report only errors of this call
  int grid = (launch && launch->grid > 0) ? launch->grid : (n_units + waves - 1) / waves;
  if (grid < 1) grid = 1;
  if (!(launch && launch->grid > 0) && grid > 8192) grid = 8192;
  const int count_block = 256, count_waves = count_block / kWave;
  int count_grid = (n_units + count_waves - 1) / count_waves;
  if (count_grid > 8192) count_grid = 8192;
  if (count_grid < 1) count_grid = 1;
  const size_t count_lds = (size_t)count_waves * (S + 1) * sizeof(uint32_t);
  if (n_units > 0) {
    if (!allow_dynamic_lds(reinterpret_cast<const void*>(k_decode_count), count_lds) ||
        !allow_dynamic_lds(reinterpret_cast<const void*>(k_decode), lds))
      return UTC_ERR_HIP;
    hipLaunchKernelGGL(k_decode_count, dim3(count_grid), dim3(count_block), count_lds, stream, g,
                       words, bank_offsets, n_units, unit_sum, error_flags);
  }
  hipLaunchKernelGGL(k_decode_scan, dim3(1), dim3(1024), 0, stream, unit_sum, n_units, unit_base,
                     hit_offsets + (int64_t)n_units * S);
  if (n_units > 0) {
    HitsOut out{lhcbid, z, u, y_begin, y_end, weight};
    hipLaunchKernelGGL(k_decode, dim3(grid), dim3(block), lds, stream, g, words, bank_offsets,
                       n_units, cap, hit_capacity, unit_base, hit_offsets, out, error_flags);
  }
  return hipGetLastError() == hipSuccess ? UTC_OK : UTC_ERR_HIP;
}

// Host-side argument checks shared by ut_decode and ut_decode_noalloc.
static bool decode_args_ok(const utc_geometry* geom, const uint16_t* words,
                           const uint32_t* bank_offsets, int32_t n_events, int64_t hit_capacity,
                           const uint32_t* hit_offsets, const uint32_t* lhcbid, const float* u,
                           const float* weight, const utc_launch_config* launch)
{
  if (!geom || geom->n_layers != kLayers || geom->n_sectors < 1 || geom->n_sectors > 8192 ||
      !geom->u0 || n_events < 0 || hit_capacity < 0 || !bank_offsets || !hit_offsets)
    return false;
  if (n_events > 0 && hit_capacity > 0 && (!words || !lhcbid || !u || !weight)) return false;
  if (launch && (launch->block < 64 || launch->block > 1024 || launch->block % 64 || launch->grid < 0 ||
                 launch->window_tile < 0 || launch->window_tile > 40 ||
                 (launch->window_tile > 0 && launch->window_tile < 4)))
    return false;
  if ((int64_t)n_events * kLayers > INT32_MAX / 2) return false;
  return true;
}

extern "C" utc_status ut_decode(const utc_geometry* geom, const uint16_t* words,
                                const uint32_t* bank_offsets, int32_t n_events, int64_t hit_capacity,
                                uint32_t* hit_offsets, uint32_t* lhcbid, float* z, float* u,
                                float* y_begin, float* y_end, float* weight, uint32_t* error_flags,
                                void* workspace, size_t workspace_bytes,
                                const utc_launch_config* launch, hipStream_t stream)
{
  if (!decode_args_ok(geom, words, bank_offsets, n_events, hit_capacity, hit_offsets, lhcbid, u,
                      weight, launch))
    return UTC_ERR_ARG;
  const size_t need = ut_decode_workspace_bytes(n_events, geom->n_sectors);
  if (!workspace || workspace_bytes < need) return UTC_ERR_WORKSPACE;
  return decode_launch(geom, words, bank_offsets, n_events, hit_capacity, hit_offsets, lhcbid, z, u,
                       y_begin, y_end, weight, error_flags, static_cast<uint32_t*>(workspace),
                       launch, stream);
}

// ---- ut_decode without a workspace argument ----
// The unit sums and bases live in a fixed device array of the library (one copy per GPU, held
// until the process ends).  In host code `scratch` names a host-side stand-in, not the device
// copy: kernels get the address hipGetSymbolAddress returns for the current device.
constexpr size_t kNoAllocScratchWords = 2 * (size_t)UTC_NOALLOC_MAX_EVENTS * kLayers + 1;
static __device__ __align__(256) uint32_t scratch[kNoAllocScratchWords];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
uint32_t* g_scratch_ptr[kMaxDevices] = {};   // device address of `scratch`, per device

// Address of the calling device's `scratch`, looked up once per device (with that device
// current); nullptr when HIP reports an error.
uint32_t* device_scratch()
{
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
    (void)hipGetLastError();
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch_ptr[dev] = static_cast<uint32_t*>(p);
  }
  return g_scratch_ptr[dev];
}
}  // namespace

extern "C" utc_status ut_decode_noalloc(const utc_geometry* geom, const uint16_t* words,
                                        const uint32_t* bank_offsets, int32_t n_events,
                                        int64_t hit_capacity, uint32_t* hit_offsets,
                                        uint32_t* lhcbid, float* z, float* u, float* y_begin,
                                        float* y_end, float* weight, uint32_t* error_flags,
                                        const utc_launch_config* launch, hipStream_t stream)
{
  if (!decode_args_ok(geom, words, bank_offsets, n_events, hit_capacity, hit_offsets, lhcbid, u,
                      weight, launch))
    return UTC_ERR_ARG;
  if (n_events > UTC_NOALLOC_MAX_EVENTS) return UTC_ERR_ARG;
  uint32_t* ws = device_scratch();
  if (!ws) return UTC_ERR_HIP;
  return decode_launch(geom, words, bank_offsets, n_events, hit_capacity, hit_offsets, lhcbid, z, u,
                       y_begin, y_end, weight, error_flags, ws, launch, stream);
}
