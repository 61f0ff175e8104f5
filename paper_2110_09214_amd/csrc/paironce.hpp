// Pair-once evaluation of pairwise sums (targets = sources): ownership of
// super-block pairs and the rule that leaves tile pairs to the directed
// kernels, shared by the field and its adjoint.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace obem {

// Number of partners d = 1 .. sym_h(A) that super-block A owns among ns:
// A owns (A, A + d mod ns), so that every unordered pair of super-blocks has
// one owner and the owners' shares differ by at most one.
__host__ __device__ __forceinline__ int sym_h(int A, int ns) {
  return (ns & 1) ? (ns - 1) / 2 : (A < ns / 2 ? ns / 2 : ns / 2 - 1);
}

// Squared gap between the boxes of source tiles a and b (FP64, 256-source
// tiles), symmetric in a and b bit for bit.
__device__ __forceinline__ double tiles_gap2(const double *__restrict__ tbox, int a, int b) {
  const double *p = tbox + 6 * (size_t)a, *q = tbox + 6 * (size_t)b;
  double g2 = 0.0;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const double g = fmax(0.0, fmax(q[c] - p[3 + c], p[c] - q[3 + c]));
    g2 = fma(g, g, g2);
  }
  return g2;
}

// Whether the tile pair (a, b) is left to the directed kernel under the
// pair-once evaluation (super-blocks of sym_tiles tiles): tiles of one
// super-block, tiles within the partner cut (nn), and tiles closer than an
// eighth of the smaller radius R of their two super-blocks (sb: centre and
// R^2 per super-block).  The pair-once kernels recentre a super-block pair
// on the centre of the super-block with the smaller radius
// (sym_origin), so beyond that gap the FP32 difference r - s they form, from
// coordinates of size up to R + |r - s|, carries at most about 17 ulps of
// |r - s|.  Symmetric in a and b, and evaluated the same way by both sides,
// so that every tile pair is taken by exactly one of them.
__device__ __forceinline__ bool tile_pair_direct(const double *__restrict__ tbox, const double *__restrict__ sb,
                                                 int a, int b, int sym_tiles, bool nn, double cut2) {
  const int A = a / sym_tiles, B = b / sym_tiles;
  if (A == B) return true;
  const double g2 = tiles_gap2(tbox, a, b);
  return 64.0 * g2 < fmin(sb[4 * (size_t)A + 3], sb[4 * (size_t)B + 3]) || (nn && g2 <= cut2);
}

// The origin of the super-block pair (A, B): the centre of the one with the
// smaller radius (A on a tie).
__device__ __forceinline__ const double *sym_origin(const double *__restrict__ sb, int A, int B) {
  return sb[4 * (size_t)B + 3] < sb[4 * (size_t)A + 3] ? sb + 4 * (size_t)B : sb + 4 * (size_t)A;
}

// Work item (A, dd) of workgroup w of a pair-once launch over ns super-blocks
// and dcnt values of d, in a one-dimensional grid of nw = sym_grid(ns, dcnt)
// workgroups.  The chip deals workgroups to its 8 XCDs in turn (w mod 8), and
// each XCD has an L2 of its own, so item t = (w mod 8) (nw / 8) + w / 8 gives
// every XCD a contiguous run of items.  Items run over A within bands of 16
// values of d (d fastest), so the 256 workgroups an XCD holds at once share
// 16 super-blocks A and about 31 super-blocks B in its L2 instead of reading
// 256 of each.  Returns false for the few padding workgroups beyond
// ns x dcnt.  Any order gives the same result (each workgroup writes its own
// slots); the order only sets what the L2 can reuse.
constexpr int kSymXcds = 8;
constexpr int kSymBand = 16;

inline unsigned sym_grid(int ns, int dcnt) {
  const long long t = (long long)ns * dcnt;
  return (unsigned)((t + kSymXcds - 1) / kSymXcds * kSymXcds);
}

__device__ __forceinline__ bool sym_item(int ns, int dcnt, int &A, int &dd) {
  const int w = (int)blockIdx.x, nw = (int)gridDim.x;
  const int t = (w % kSymXcds) * (nw / kSymXcds) + w / kSymXcds;
  if (t >= ns * dcnt) return false;
  const int band = t / (ns * kSymBand);
  const int bw = min(kSymBand, dcnt - band * kSymBand);
  const int r = t - band * ns * kSymBand;
  A = r / bw;
  dd = band * kSymBand + r % bw;
  return true;
}

// Workgroups of `kernel` (blocks of `threads`) resident at once on `device`,
// or 1 if the runtime cannot tell.
inline int resident_workgroups(const void *kernel, int threads, int device) {
  int per_cu = 0, cus = 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, threads, 0) != hipSuccess || per_cu < 1 ||
      cus < 1) {
    (void)hipGetLastError();
    return 1;
  }
  return per_cu * cus;
}

// Values of d for the next pair-once launch: all remaining if they fit in
// max_slots, else the count in [max_slots / 2, max_slots] whose ns x count
// equal workgroups leave the smallest share of the launch's last round of
// resident workgroups idle.
inline int launch_slots(int ns, int remaining, int resident, int max_slots) {
  if (remaining <= max_slots || resident <= 1) return remaining < max_slots ? remaining : max_slots;
  int best = max_slots;
  double best_waste = 2.0;
  for (int c = max_slots; c >= max_slots / 2; --c) {
    const long long items = (long long)ns * c;
    const long long idle = (resident - items % resident) % resident;
    const double waste = (double)idle / (double)items;
    if (waste < best_waste - 1e-12) {
      best_waste = waste;
      best = c;
    }
  }
  return best;
}

}  // namespace obem
