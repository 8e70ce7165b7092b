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
