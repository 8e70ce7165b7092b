// Sparse pore-site lattice and int32 pull table (host side).
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

namespace flbm {

struct LatticeSpec {
    int nx = 0, ny = 0, nz = 0;
    int periodic_x = 1, periodic_y = 1;
    int z_mode = 0;  // FLBM_Z_*
    int reservoir_layers = 0;
};

// Pore sites in raster order (z slowest, x fastest) and, for each site s and
// direction q = 1..18, the flat index into a [19][n_pad] distribution array
// of the value that streams into (q, s):
//   q*n_pad + src        source pore site x_s - xi_q,
//   opp(q)*n_pad + s     halfway bounce-back (source solid or beyond a
//                        non-periodic side, or beyond z in wall mode),
//   sentinel             source beyond z = 0 or z = nz-1 in flux mode: a
//                        boundary unknown (Methods, the definition of the
//                        unknowns before eq. inlet); the sentinel addresses a
//                        zero slot past the 19 rows.
struct Lattice {
    int64_t n = 0, n_pad = 0, a_in = 0, a_out = 0;
    int64_t n01 = 0;              // sites of planes z = 0 and z = 1
    int64_t sentinel = 0;
    std::vector<int32_t> coords;  // [n][3]
    std::vector<int32_t> nbr;     // [18][n_pad], row q-1 for direction q
    // Flux mode: for each site of planes 0-1, bits 2q..2q+1 hold the weight
    // (0, 1 or 2) with which its stored population q enters the next step's
    // inlet consistency sum (eq. inlet: 1 for in-plane, 2 for populations
    // leaving through the inlet; the pull table maps each such population to
    // exactly one inlet site and direction).
    std::vector<uint64_t> kcoef;  // [n01]
};

// Compact forms of the pull table (see pull_format.h) for tiles of `tile`
// sites: 16-bit codes [9][n_pad], byte codes [4][n_pad] + [n_pad], and a
// PULL_HDR-int32 header per tile. Rows of a tile in another form are zero.
struct CompactPull {
    int tile = 0;
    int32_t limit16 = 0, limit8 = 0;  // largest regular code of each form (0: form not used)
    int64_t tiles = 0, tiles16 = 0, tiles8 = 0;
    int64_t tiles_run = 0, waves_wide = 0;  // byte tiles with run codes; their waves listing > 256 codes
    std::vector<uint32_t> codes;   // [9][n_pad] 16-bit codes
    std::vector<uint32_t> bytes;   // [4][n_pad] byte codes of directions 1..16
    std::vector<uint16_t> tail;    // [n_pad] byte codes of directions 17 (low) and 18 (high)
    std::vector<uint32_t> runs;    // [n_pad][2] run codes: mask, list bytes 4l..4l+3
    std::vector<uint32_t> runs_hi; // [n_pad] list bytes 256+4l..256+4l+3
    std::vector<int32_t> hdr;      // [tiles][PULL_HDR]
};

// Builds the compact forms of L's pull table for tiles of `tile` sites
// (n_pad must be a multiple): each tile takes byte codes if its sources fit
// limit8 (0 <= limit8 <= PULL_MAX_BYTE; 0 turns byte codes off), else
// 16-bit codes if they fit limit16 (1 <= limit16 <= PULL_MAX_CODE), else
// the int32 table. Byte tiles whose waves all list at most PULL_RUN_MAX
// codes also get run codes (see pull_format.h) and the header's run flag.
// Returns "" on success.
std::string build_compact_pull(const Lattice &L, int tile, int32_t limit16, int32_t limit8, CompactPull &out);

// Every entry of every coded tile decodes to the int32 table's entry, and
// every row of a tile in another form is zero. Returns "" if it holds.
std::string check_compact_pull(const Lattice &L, const CompactPull &cp);

// Row length of every [q][site] array: a multiple of 1024 sites.
int64_t padded_sites(int64_t n);

// Builds the lattice. Returns an empty string on success, else an error text.
// `code` receives an flbm_status on failure.
std::string build_lattice(const uint8_t *solid, const LatticeSpec &spec, Lattice &out, int &code);

// Structural race check: every slot (q, s) of the source array is read by at
// most one (q', s') of the pull table, and the slots never read are exactly
// the populations that leave through the z faces. Returns "" if it holds.
std::string check_pull_bijection(const Lattice &L, const LatticeSpec &spec);

}  // namespace flbm
