// The persistent drain kernel (flix_drain.hpp) in a translation unit of its
// own, instantiated for both key widths, both digit widths and every
// lane-group shape the autotuner sweeps.
#include <algorithm>

#include "flix_launch.hpp"

namespace flix {
namespace {

template <typename K, int RB, int GL, int KPL>
hipError_t drain_t(const DrainLaunch& d, hipStream_t st) {
  size_t shm = DrainSmemSize<K, RB, GL, KPL>::fixed();
  const size_t upd = (size_t)(256 / GL) * 2 * d.lds_items * sizeof(K);
  if (upd > shm) shm = upd;
  auto kfn = k_drain<K, RB, GL, KPL>;
  hipError_t e;
  if (*d.grid == 0 || *d.shm != shm) {
    if (shm > 65536 &&
        (e = hipFuncSetAttribute(reinterpret_cast<const void*>(kfn),
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm)) != hipSuccess)
      return e;
    int per_cu = 0, dev = 0, cus = 0;
    if ((e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kfn, 256, shm)) != hipSuccess ||
        (e = hipGetDevice(&dev)) != hipSuccess ||
        (e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess)
      return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    // At most two workgroups per CU: every batch pays several grid barriers,
    // whose cost grows with the arrivals; measured on the mixed-batch stream,
    // two per CU beat three (540 vs 475 Mops/s) and one (537, slower on large
    // batches).
    *d.grid = std::min(per_cu, 2) * cus;
    *d.shm = shm;
  }
  DrainArgs<K> a;
  a.batches = d.batches;
  a.nbatch = d.nbatch;
  a.layout = d.layout;
  a.cap = d.cap;
  a.ctl = d.ctl;
  a.bk[0] = (K*)d.bk[0];
  a.bk[1] = (K*)d.bk[1];
  a.bp[0] = d.bp[0];
  a.bp[1] = d.bp[1];
  a.hist = d.hist;
  a.status = d.status;
  a.status_cl = d.status_cl;
  a.status_words = d.status_words;
  a.cluster_words = d.cluster_words;
  a.work = d.work;
  a.lds_items = d.lds_items;
  a.chunk = d.chunk;
  a.dctl = d.dctl;
  a.tstamp = d.tstamp;
  a.max_batch = d.max_batch;
  hipLaunchKernelGGL(kfn, dim3(*d.grid), dim3(256), shm, st, a);
  return hipGetLastError();
}

template <typename K, int RB>
hipError_t drain_rb(const DrainLaunch& d, hipStream_t st) {
  const u32 kpl = std::max<u32>(1u, d.cap / d.gl);
  switch (d.gl * 100 + kpl) {
    case 1601: return drain_t<K, RB, 16, 1>(d, st);
    case 1602: return drain_t<K, RB, 16, 2>(d, st);
    case 1604: return drain_t<K, RB, 16, 4>(d, st);
    case 1608: return drain_t<K, RB, 16, 8>(d, st);
    case 1616: return drain_t<K, RB, 16, 16>(d, st);
    case 3201: return drain_t<K, RB, 32, 1>(d, st);
    case 3202: return drain_t<K, RB, 32, 2>(d, st);
    case 3204: return drain_t<K, RB, 32, 4>(d, st);
    case 3208: return drain_t<K, RB, 32, 8>(d, st);
    case 6401: return drain_t<K, RB, 64, 1>(d, st);
    case 6402: return drain_t<K, RB, 64, 2>(d, st);
    default: return drain_t<K, RB, 64, 4>(d, st);
  }
}

}  // namespace

hipError_t drain_launch(const DrainLaunch& d, hipStream_t st) {
  if (d.key_bits == 32)
    return d.radix_bits == 4 ? drain_rb<u32, 4>(d, st) : drain_rb<u32, 8>(d, st);
  return d.radix_bits == 4 ? drain_rb<u64, 4>(d, st) : drain_rb<u64, 8>(d, st);
}

}  // namespace flix
