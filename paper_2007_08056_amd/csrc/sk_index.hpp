// Work partition of the stream-K sector product, shared by its kernels, its
// launcher and the host-side replay that checks it: which K-iterations each
// persistent workgroup takes, where it leaves the pieces of the tiles it cuts,
// and which pieces the fixup sums for each tile.
//
// Tiles come in groups of `ts` (1, or the tiles_n tiles of one (q, M-panel),
// which read the same A rows).  A team of ts workgroups, one per tile of a
// group, owns the K-iterations [bound(t), bound(t + 1)) of the concatenation of
// all groups (group-major, nk iterations each): its members walk the same
// groups and K-steps side by side, so each A panel is fetched into L2 once per
// team rather than once per tile.  Workgroups are dispatched round-robin over
// the 8 XCDs, so workgroup b is slot b / 8 on XCD b % 8, and the teams of one
// XCD hold consecutive shares.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace symt {

// First K-iteration of team t's share: total iterations split as evenly as integers allow.
__host__ __device__ inline int64_t sk_bound(int64_t t, int64_t total, int nteam) {
  return t * total / nteam;
}

// Team, member and team count of persistent workgroup b of a launch of `grid`
// workgroups (grid = 8 * teams_x * ts).
struct SkSlot {
  int team, member, nteam;
};
__host__ __device__ inline SkSlot sk_slot(int b, int grid, int ts) {
  const int teams_x = grid / (8 * ts);
  const int l = b / 8;                          // slot on this XCD
  return SkSlot{(b % 8) * teams_x + l / ts, l % ts, 8 * teams_x};
}

// Piece buffer index of the piece that (team, member) leaves for group `grp`:
// two per workgroup, the first for the group its share starts in, the second
// for the group it ends in (a share that spans whole groups cuts at most those two).
__host__ __device__ inline int64_t sk_piece(int team, int member, int ts, int64_t grp, int64_t first_grp) {
  return 2 * (static_cast<int64_t>(team) * ts + member) + (grp == first_grp ? 0 : 1);
}

// Last team whose share starts at or before iteration x0 (the first team that
// holds part of the group starting at x0).
__host__ __device__ inline int64_t sk_first_team(int64_t x0, int64_t total, int nteam) {
  return ((x0 + 1) * nteam - 1) / total;
}

// Host side: persistent workgroups and team width of a stream-K launch.
// `resident`: workgroups the device holds at once (CUs x occupancy, capped);
// `part_elems`: elements the pieces buffer holds; `tile_elems`: BM * BN.
// Returns P = 0 when stream-K does not pay (too few iterations per team) or
// the buffer is too small; then the product runs one workgroup per tile.
struct SkLaunch {
  int P = 0;      // persistent workgroups (a multiple of 8 * ts)
  int ts = 1;     // team width
};
inline SkLaunch sk_launch(int64_t ntiles, int tiles_n, int nk, int64_t resident, int64_t part_elems,
                          int64_t tile_elems, int min_iters) {
  SkLaunch out;
  const int64_t fit = part_elems / (2 * tile_elems);
  const int64_t slots = resident < fit ? resident : fit;
  // teams of tiles_n siblings when 8 XCDs hold at least one team each
  const int64_t per_xcd = slots / 8;
  const int ts = tiles_n <= per_xcd ? tiles_n : 1;
  int64_t teams_x = per_xcd / ts;
  const int64_t by_work = (ntiles / ts) * nk / min_iters;   // teams with >= min_iters each
  if (by_work / 8 < teams_x) teams_x = by_work / 8;
  const int64_t P = 8 * teams_x * ts;
  if (P < 8 || 2 * P * tile_elems > part_elems) return out;
  out.P = static_cast<int>(P);
  out.ts = ts;
  return out;
}

}  // namespace symt
