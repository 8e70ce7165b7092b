// Compact forms of the pull table, shared by the host builder and the step
// kernel.
//
// Within one tile of consecutive sites (sites in raster order), the sources
// that stream into a fixed direction q lie in a narrow range of site numbers:
// the tile's own range shifted by the direction's raster offset, widened at
// most by a wrap across a periodic side. Each tile takes the narrowest of
// three forms that holds all its sources:
//
// byte codes (PULL_TILE_BYTE): per direction a base, per site and direction
//   an 8-bit code c against the site's position p in the tile:
//     0 .. PULL_MAX_BYTE   regular source: flat index = base + p + c
//     PULL_BYTE_UNKNOWN    boundary unknown: the sentinel (zero slot)
//     PULL_BYTE_BOUNCE     halfway bounce-back: opp(q) * n_pad + site
//   (in a pore region the source runs along with the site, so c stays small
//   while the site numbers themselves drift); directions 1..16 in four
//   words [4][n_pad] (byte j of word k is direction 4k+j+1), 17 and 18 in a
//   16-bit row [n_pad]: 18 bytes per site;
// 16-bit codes (PULL_TILE_HALF): c against the base alone,
//     0 .. PULL_MAX_CODE   regular source: flat index = base + c
//     PULL_UNKNOWN, PULL_BOUNCE as above;
//   directions 2k+1 (low half) and 2k+2 (high half) share word k of
//   [9][n_pad]: 36 bytes per site;
// the int32 table (PULL_TILE_INT32): 72 bytes per site, for tiles whose
//   sources of some direction span more than the 16-bit range (a y-wrap
//   across a plane wider than 65533 pore sites, or a tile stretched over a
//   nearly solid region).
//
// Run codes (header entry PULL_HDR_RUNS = 1, byte-coded tiles only): along a
// run of pore sites the byte code of a direction stays the same from site to
// site (source and site advance together) and changes only where the solid
// structure interrupts a run, at about one site in six. Each wave of 64
// consecutive sites (one per lane) then keeps, per site, a mask of the
// directions whose code differs from the previous site's (bit q-1; every
// direction at the wave's first site), and the wave's list of those codes,
// direction by direction and in site order within a direction. The list is
// held four bytes per lane: bytes 4l..4l+3 in word 1 of lane l's record
// [n_pad][2] (word 0: the mask, bit 31 set on every lane when the list is
// longer than 256 bytes), bytes 256+4l..256+4l+3 in a second row [n_pad]. A
// site's code of direction q is entry off_q + r of the list, off_q the
// number of listed codes of the directions before q and r the number of
// listed codes of q at the site's lane and below, minus one. A tile takes
// run codes when every one of its waves lists at most 512 codes: 8 bytes per
// site (12 where a list is longer than 256 bytes) instead of 18.
#pragma once
#include <stdint.h>

namespace flbm {

constexpr int PULL_HDR = 20;          // int32 per tile: 18 bases, the tile's form, the run flag
constexpr int PULL_HDR_FORM = 18;
constexpr int PULL_HDR_RUNS = 19;
constexpr int PULL_RUN_WAVE = 64;     // sites of a wave of run codes
constexpr int PULL_RUN_MAX = 512;     // listed codes per wave at most
constexpr uint32_t PULL_RUN_WIDE = 1u << 31;  // mask bit: the wave's list exceeds 256 bytes
constexpr int PULL_TILE_INT32 = 0;
constexpr int PULL_TILE_HALF = 1;
constexpr int PULL_TILE_BYTE = 2;
constexpr uint32_t PULL_BOUNCE = 0xFFFFu;
constexpr uint32_t PULL_UNKNOWN = 0xFFFEu;
constexpr uint32_t PULL_MAX_CODE = 0xFFFDu;
constexpr uint32_t PULL_BYTE_BOUNCE = 0xFFu;
constexpr uint32_t PULL_BYTE_UNKNOWN = 0xFEu;
constexpr uint32_t PULL_MAX_BYTE = 0xFDu;

}  // namespace flbm
