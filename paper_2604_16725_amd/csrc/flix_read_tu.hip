// Read kernels of the C ABI, in a translation unit of their own: the
// sorted-share kernel (flix_read2.hpp) and the bucket-group kernel
// (flix_group.hpp), instantiated for every lane-group shape.
#include <algorithm>

#include "flix_launch.hpp"
#include "flix_sort.hpp"

namespace flix {
namespace {

template <typename K>
struct ReadShare {
  static constexpr int S = 512;   // merged items (buckets + keys) per workgroup
};

template <typename K, int GL, int KPL>
void read2_k(const ReadArgs<K>& a, int op, u32 grid, hipStream_t st, hipEvent_t e0,
             hipEvent_t e1) {
  // One bucket per lane group at a time: the eight resident waves per SIMD
  // keep enough node loads in flight, and the registers of more buckets cost
  // spills or occupancy (lookup / successor / range16 kernels on a 2^26-key
  // store: 69 / 87 / 98 us holding two to four buckets, 64 / 84 / 95 us
  // holding one).
  constexpr int U = 1;
  constexpr int S = ReadShare<K>::S;
  switch (op) {
    case kOpLookup:
      launch_timed(e0, e1, k_read_apply2<K, 256, S, GL, KPL, U, kOpLookup>, dim3(grid), dim3(256),
                   0, st, a);
      break;
    case kOpSuccessor:
      launch_timed(e0, e1, k_read_apply2<K, 256, S, GL, KPL, U, kOpSuccessor>, dim3(grid),
                   dim3(256), 0, st, a);
      break;
    case kOpRange:
      launch_timed(e0, e1, k_read_apply2<K, 256, S, GL, KPL, U, kOpRange>, dim3(grid), dim3(256),
                   0, st, a);
      break;
    default:
      launch_timed(e0, e1, k_read_apply2<K, 256, S, GL, KPL, U, kOpPredecessor>, dim3(grid),
                   dim3(256), 0, st, a);
      break;
  }
}

// U buckets in a lane group's registers at a time.
template <typename K, int GL, int KPL>
void group_k(const GroupArgs<K>& ga, const ReadArgs<K>& a, int op, u32 grid, hipStream_t st,
             hipEvent_t e0, hipEvent_t e1) {
  constexpr int KW = KPL * (int)(sizeof(K) / 4);
  constexpr int U = KW >= 16 ? 2 : 4;
  auto fn = k_group_read<K, 256, 8, GL, KPL, U>;
  const GroupLds<K> L(2048, 256, kGroupBucketsMax, op == kOpRange);
  static size_t attr = 0;
  if (L.bytes > 65536 && L.bytes > attr) {
    if (hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.bytes) == hipSuccess)
      attr = L.bytes;
    (void)hipGetLastError();
  }
  launch_timed(e0, e1, fn, dim3(grid), dim3(256), (uint32_t)L.bytes, st, ga, a, op);
}

}  // namespace

// Lanes per bucket GL and keys per lane KPL = max(1, cap / GL).
template <typename K>
void launch_read2(u32 gl, u32 cap, const ReadArgs<K>& a, int op, u32 grid, hipStream_t st,
                  hipEvent_t e0, hipEvent_t e1) {
  const u32 kpl = std::max<u32>(1u, cap / gl);
  switch (gl * 100 + kpl) {
    case 1601: read2_k<K, 16, 1>(a, op, grid, st, e0, e1); break;
    case 1602: read2_k<K, 16, 2>(a, op, grid, st, e0, e1); break;
    case 1604: read2_k<K, 16, 4>(a, op, grid, st, e0, e1); break;
    case 1608: read2_k<K, 16, 8>(a, op, grid, st, e0, e1); break;
    case 1616: read2_k<K, 16, 16>(a, op, grid, st, e0, e1); break;
    case 3201: read2_k<K, 32, 1>(a, op, grid, st, e0, e1); break;
    case 3202: read2_k<K, 32, 2>(a, op, grid, st, e0, e1); break;
    case 3204: read2_k<K, 32, 4>(a, op, grid, st, e0, e1); break;
    case 3208: read2_k<K, 32, 8>(a, op, grid, st, e0, e1); break;
    case 6401: read2_k<K, 64, 1>(a, op, grid, st, e0, e1); break;
    case 6402: read2_k<K, 64, 2>(a, op, grid, st, e0, e1); break;
    default: read2_k<K, 64, 4>(a, op, grid, st, e0, e1); break;
  }
}

template <typename K>
void launch_group(u32 gl, u32 cap, const GroupArgs<K>& ga, const ReadArgs<K>& a, int op,
                  u32 grid, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  const u32 kpl = std::max<u32>(1u, cap / gl);
  switch (gl * 100 + kpl) {
    case 1601: group_k<K, 16, 1>(ga, a, op, grid, st, e0, e1); break;
    case 1602: group_k<K, 16, 2>(ga, a, op, grid, st, e0, e1); break;
    case 1604: group_k<K, 16, 4>(ga, a, op, grid, st, e0, e1); break;
    case 1608: group_k<K, 16, 8>(ga, a, op, grid, st, e0, e1); break;
    case 1616: group_k<K, 16, 16>(ga, a, op, grid, st, e0, e1); break;
    case 3201: group_k<K, 32, 1>(ga, a, op, grid, st, e0, e1); break;
    case 3202: group_k<K, 32, 2>(ga, a, op, grid, st, e0, e1); break;
    case 3204: group_k<K, 32, 4>(ga, a, op, grid, st, e0, e1); break;
    case 3208: group_k<K, 32, 8>(ga, a, op, grid, st, e0, e1); break;
    case 6401: group_k<K, 64, 1>(ga, a, op, grid, st, e0, e1); break;
    case 6402: group_k<K, 64, 2>(ga, a, op, grid, st, e0, e1); break;
    default: group_k<K, 64, 4>(ga, a, op, grid, st, e0, e1); break;
  }
}

// The library builds this file once per key width (FLIX_READ_KEY_BITS = 32 or
// 64), so the two halves of the read kernels compile in parallel.
#if FLIX_READ_KEY_BITS == 32
template void launch_read2<u32>(u32, u32, const ReadArgs<u32>&, int, u32, hipStream_t, hipEvent_t,
                                hipEvent_t);
template void launch_group<u32>(u32, u32, const GroupArgs<u32>&, const ReadArgs<u32>&, int, u32,
                                hipStream_t, hipEvent_t, hipEvent_t);
#elif FLIX_READ_KEY_BITS == 64
template void launch_read2<u64>(u32, u32, const ReadArgs<u64>&, int, u32, hipStream_t, hipEvent_t,
                                hipEvent_t);
template void launch_group<u64>(u32, u32, const GroupArgs<u64>&, const ReadArgs<u64>&, int, u32,
                                hipStream_t, hipEvent_t, hipEvent_t);
#else
#error "FLIX_READ_KEY_BITS must be 32 or 64"
#endif

}  // namespace flix
