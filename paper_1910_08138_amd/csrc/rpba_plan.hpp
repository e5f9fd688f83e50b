// Host-side planning of the device data layout (done once per problem).
//
// Orders (paper Sec. 4: every camera belongs to exactly one sub-block; a point
// may appear in several, as a "copy" per sub-block):
//   * cameras: grouped by sub-block (stable in the original index);
//   * points: by the lowest sub-block that sees them, then original index;
//   * observations ("LM order"): by (sub-block, point, camera), so that every
//     copy (sub-block, point) is one contiguous run of observations and the
//     copies of one sub-block are contiguous.
// The same order serves the intersection (a point visits its copies) and the
// sub-block step (a sub-block visits its copies).
#pragma once
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

namespace rpba {

constexpr int INT_WG = 128;        // points per intersection workgroup
constexpr int INT_CAM_CAP = 192;   // cameras staged in LDS per intersection workgroup
constexpr int INT_OBS_CAP = 768;   // observations staged in LDS per intersection workgroup
constexpr int PB_LANES = 8;        // lanes per off-diagonal pair block in the pair Schur pass
// intersection observation code: camera slot in the workgroup's LDS list, or
// with PM_GLOBAL the camera index itself; PM_DOWN = robust down-weighting,
// with PM_DEL as well = deleted (weight 0); PM_LAST = last observation of its
// copy (the copies of a point follow each other in the stream)
constexpr int32_t PM_DEL = 1 << 27;
constexpr int32_t PM_LAST = 1 << 28;
constexpr int32_t PM_GLOBAL = 1 << 29;
constexpr int32_t PM_DOWN = 1 << 30;
constexpr int32_t PM_FIELD = PM_DEL - 1;

struct Plan {
  int32_t M = 0, N = 0, K = 0, L = 0;
  int64_t NC = 0;  // copies
  int32_t T = 64;  // Cholesky tile edge
  int32_t np = 6;  // parameters per camera (RCS rows per camera): 6, or 8 with intrinsics
  bool has_info = false;

  // permutations (new -> original)
  std::vector<int32_t> cam_orig, pt_orig, obs_orig;
  std::vector<int32_t> pt_new;         // [N] internal index of caller point o
  std::vector<int32_t> cam_blk;        // [M] sub-block of internal camera
  std::vector<int32_t> blk_cam_off;    // [L+1]
  std::vector<int32_t> obs_cam;        // [K] internal camera of LM-ordered observation
  std::vector<int32_t> obs_copy;       // [K]
  std::vector<int32_t> copy_off;       // [NC+1] observation runs
  std::vector<int32_t> copy_pt;        // [NC] internal point
  std::vector<int32_t> copy_blk;       // [NC]
  std::vector<int64_t> blk_copy_off;   // [L+1]
  std::vector<int32_t> pt_copy_off;    // [N+1]
  std::vector<int32_t> pt_copies;      // [NC] copy indices grouped by point (ascending sub-block)
  // intersection stream (point-major): the observations of point j at
  // [pm_off[j], pm_off[j+1]), copy by copy in pt_copies order; each launch
  // workgroup of INT_WG points stages its observations (at most INT_OBS_CAP)
  // and the cameras they see (at most INT_CAM_CAP) in LDS: pm_cam is the
  // camera's slot there, or PM_GLOBAL | camera
  std::vector<int32_t> pm_off;         // [N+1]
  std::vector<int32_t> pm_k;           // [K] LM index
  std::vector<int32_t> pm_pos;         // [K] position of LM index k
  std::vector<int32_t> pm_cam;         // [K]
  std::vector<int32_t> iwg_cam_off;    // [ceil(N / INT_WG) + 1]
  std::vector<int32_t> iwg_cams;       // internal camera indices
  std::vector<int32_t> cam_obs_off;    // [M+1]
  std::vector<int32_t> cam_obs;        // [K] LM-ordered observation indices per camera
  std::vector<int32_t> cam_obs_c;      // [K] copy of each entry of cam_obs
  std::vector<int32_t> nb_off;         // [M+1] neighbour lists (cameras of the same
  std::vector<int32_t> nb_cam;         //        sub-block sharing a point, local index <= own)
  int32_t max_nb = 0, max_blk_cams = 0, max_cam_obs = 0;
  // pair blocks = neighbour entries: block (i, nb_cam[q]) of the RCS of camera
  // i's sub-block, with the observation pairs (k1 of camera i, k2 of the
  // neighbour, same copy) that contribute to it
  std::vector<int32_t> pb_row;         // [NPB] internal camera i
  std::vector<int64_t> pb_ent_off;     // [NPB+1]
  std::vector<int32_t> pb_ent;         // [3 * entries] (copy, t1, t2): t = the observation's position in cam_obs
  std::vector<int32_t> od_pb;          // off-diagonal pair blocks (i2 != i), most lane-group rounds first
  std::vector<int32_t> pb_bsr;         // [NPB] position of block (i, i2) in the full block-sparse matrix
  std::vector<int32_t> pb_bsr_t;       // [NPB] position of block (i2, i)

  // dense reduced camera systems (tile-major lower triangle per sub-block)
  std::vector<int32_t> nt;             // [L] tiles per side
  std::vector<int64_t> rcs_off;        // [L] offset (doubles) of tile (0,0)
  std::vector<int64_t> diag_off;       // [L] offset of the nt factor/inverse diagonal tiles
  std::vector<int64_t> vec_off;        // [L] offset of the padded vectors
  int64_t rcs_total = 0, diag_total = 0, vec_total = 0;
  int32_t nt_max = 0;
  // [rcs_total / T^2] 1 = the tile may be nonzero in the Cholesky factor
  // (tiles numbered like the storage: sub-block l's tile (i, j) is tile
  // rcs_off[l] / T^2 + i (i + 1) / 2 + j); a zero tile keeps the zeros of S
  std::vector<uint8_t> tile_nz;
  // Cholesky work lists: item = (l << 16) | (i << 8) | j.  Tile row nt of a
  // sub-block holds the right-hand side (row 0 = e^T), so that the forward
  // substitution is part of the factorisation.
  std::vector<int32_t> pot_items;      // step k: sub-blocks with nt > k, in [pot_off[k], pot_off[k+1])
  std::vector<int64_t> pot_off;
  std::vector<int32_t> fwd_items;      // step k: triangular solves (l, i, k), k < i <= nt
  std::vector<int64_t> fwd_off;
  std::vector<int32_t> upd_items;      // step k: updates (l, i, j), k < j <= i, j < nt
  std::vector<int64_t> upd_off;
  std::vector<int32_t> bwd_items;      // backward launch for step k (descending)
  std::vector<int64_t> bwd_off;

  // block-sparse RCS (6x6 blocks, both triangles) for the iterative solver
  std::vector<int32_t> bsr_row_off;    // [M+1] per internal camera
  std::vector<int32_t> bsr_col;        // local column camera of each block
  std::vector<int32_t> bsr_tr;         // index of the transposed block
  int64_t nbsr = 0;
  std::vector<uint8_t> blk_pcg;        // [L] 1 = iterative solver for this sub-block

  uint64_t key = 0;
};

// Returns an empty string on success, else the reason.
std::string build_plan(int32_t M, int32_t N, int32_t K, int32_t L, const int32_t* obs_cam, const int32_t* obs_pt,
                       const int32_t* cam_block, int32_t tile, int32_t np, Plan& P);

uint64_t topology_key(int32_t M, int32_t N, int32_t K, int32_t L, const int32_t* obs_cam, const int32_t* obs_pt,
                      const int32_t* cam_block, int32_t tile, int32_t np);

// Task list of the persistent forward factorisation: every tile (i, j),
// j <= i <= nt, j < nt, of the listed sub-blocks, packed (l << 16) | (i << 8)
// | j.  Tile (i, j) waits for the tiles (i, k) and (j, k), k < j, and for
// i > j for the diagonal tile (j, j).  A nonzero sub-diagonal tile (j, j-1)
// of the factor is solved by the task of diagonal tile j: its own task only
// sums its products, the diagonal task waits for those sums and for diagonal
// tile j-1, and every other user of tile (j, j-1) waits for diagonal task j.
// The list is a topological order of these dependencies (checked before it
// is returned: an empty list means a broken order).
// Tiles that stay zero in the factor (tile_nz) get no task, and products with
// a zero tile are left out of the sums and of the dependencies.
std::vector<int32_t> dataflow_order(const Plan& P, const std::vector<int32_t>& blocks);

}  // namespace rpba
