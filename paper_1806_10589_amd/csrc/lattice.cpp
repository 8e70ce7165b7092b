// Sparse pore-site lattice builder: solid mask -> site list + int32 pull table.
#include "lattice.h"

#include <algorithm>
#include <thread>

#include "../../include/fluxlbm.h"
#include "d3q19.h"
#include "pull_format.h"

namespace flbm {

int64_t padded_sites(int64_t n) { return ((n + 1023) / 1024) * 1024; }

namespace {

template <class F>
void parallel_for(int64_t begin, int64_t end, F &&fn)
{
    int64_t count = end - begin;
    if (count <= 0) return;
    unsigned hw = std::max(1u, std::thread::hardware_concurrency());
    int64_t nt = std::min<int64_t>(std::min<unsigned>(hw, 16u), count);
    if (nt <= 1 || count < 4) {
        fn(begin, end);
        return;
    }
    std::vector<std::thread> th;
    int64_t chunk = (count + nt - 1) / nt;
    for (int64_t t = 0; t < nt; ++t) {
        int64_t b = begin + t * chunk, e = std::min(end, b + chunk);
        if (b >= e) break;
        th.emplace_back([&fn, b, e] { fn(b, e); });
    }
    for (auto &t : th) t.join();
}

}  // namespace

std::string build_lattice(const uint8_t *solid_in, const LatticeSpec &spec, Lattice &L, int &code)
{
    const int nx = spec.nx, ny = spec.ny, nz = spec.nz;
    const int64_t plane = (int64_t)nx * ny;
    const int64_t ncell = plane * nz;
    code = FLBM_OK;

    auto is_solid = [&](int x, int y, int z) -> bool {
        if (z < spec.reservoir_layers || z >= nz - spec.reservoir_layers) return false;
        return solid_in[(int64_t)z * plane + (int64_t)y * nx + x] != 0;
    };

    // Site numbering in raster order; per-plane counts give plane offsets so
    // planes can be numbered in parallel.
    std::vector<int64_t> plane_count(nz, 0);
    parallel_for(0, nz, [&](int64_t z0, int64_t z1) {
        for (int64_t z = z0; z < z1; ++z) {
            int64_t c = 0;
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) c += !is_solid(x, y, (int)z);
            plane_count[z] = c;
        }
    });
    std::vector<int64_t> plane_off(nz + 1, 0);
    for (int z = 0; z < nz; ++z) plane_off[z + 1] = plane_off[z] + plane_count[z];
    const int64_t n = plane_off[nz];
    L.n = n;
    L.n_pad = padded_sites(n);
    L.a_in = plane_count[0];
    L.a_out = plane_count[nz - 1];
    L.n01 = plane_count[0] + plane_count[1];
    L.sentinel = 19 * L.n_pad;
    if (n == 0) {
        code = FLBM_EINVAL;
        return "the mask has no pore site";
    }
    if (spec.z_mode == FLBM_Z_FLUX && L.a_in == 0) {
        code = FLBM_ENOINLET;
        return "no pore site on the inlet plane z = 0";
    }
    // Largest index: the sentinel plus the 64-element zero pad behind it.
    if (19 * L.n_pad + 64 > (int64_t)INT32_MAX) {
        code = FLBM_EINDEX;
        return "lattice too large for 32-bit pull indices";
    }

    std::vector<int32_t> site_of;
    try {
        site_of.assign(ncell, -1);
        L.coords.assign(3 * n, 0);
        L.nbr.assign(18 * L.n_pad, 0);
    } catch (const std::bad_alloc &) {
        code = FLBM_ENOMEM;
        return "host allocation failed while building the lattice";
    }
    parallel_for(0, nz, [&](int64_t z0, int64_t z1) {
        for (int64_t z = z0; z < z1; ++z) {
            int64_t s = plane_off[z];
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    if (is_solid(x, y, (int)z)) continue;
                    site_of[z * plane + (int64_t)y * nx + x] = (int32_t)s;
                    L.coords[3 * s + 0] = x;
                    L.coords[3 * s + 1] = y;
                    L.coords[3 * s + 2] = (int32_t)z;
                    ++s;
                }
        }
    });

    const int64_t npad = L.n_pad;
    const int32_t sentinel = (int32_t)L.sentinel;
    parallel_for(0, n, [&](int64_t s0, int64_t s1) {
        for (int64_t s = s0; s < s1; ++s) {
            const int x = L.coords[3 * s], y = L.coords[3 * s + 1], z = L.coords[3 * s + 2];
            for (int q = 1; q < 19; ++q) {
                int sx = x - d3q19::cx[q], sy = y - d3q19::cy[q], sz = z - d3q19::cz[q];
                int32_t idx;
                bool bounce = false;
                if (sz < 0 || sz >= nz) {
                    if (spec.z_mode == FLBM_Z_PERIODIC) {
                        sz = (sz + nz) % nz;
                    } else if (spec.z_mode == FLBM_Z_WALL) {
                        bounce = true;
                    } else {
                        L.nbr[(q - 1) * npad + s] = sentinel;
                        continue;
                    }
                }
                if (sx < 0 || sx >= nx) {
                    if (spec.periodic_x) sx = (sx + nx) % nx;
                    else bounce = true;
                }
                if (sy < 0 || sy >= ny) {
                    if (spec.periodic_y) sy = (sy + ny) % ny;
                    else bounce = true;
                }
                if (!bounce) {
                    int32_t src = site_of[(int64_t)sz * plane + (int64_t)sy * nx + sx];
                    if (src < 0) bounce = true;
                    else idx = (int32_t)(q * npad + src);
                }
                if (bounce) idx = (int32_t)(d3q19::opp(q) * npad + s);
                L.nbr[(q - 1) * npad + s] = idx;
            }
        }
    });
    // Padding sites read their own (zero) slots so any thread may load them.
    for (int64_t s = n; s < npad; ++s)
        for (int q = 1; q < 19; ++q) L.nbr[(q - 1) * npad + s] = (int32_t)(q * npad + s);

    if (spec.z_mode == FLBM_Z_FLUX) {
        L.kcoef.assign(L.n01, 0);
        for (int64_t i = 0; i < L.a_in; ++i) {
            for (int q = 0; q < 19; ++q) {
                const int c = d3q19::inlet_coeff(q);
                if (!c) continue;
                const int64_t idx = q == 0 ? i : L.nbr[(q - 1) * npad + i];
                const int64_t qq = idx / npad, src = idx % npad;
                if (idx == L.sentinel || src >= L.n01) {
                    code = FLBM_EINVAL;
                    return "inlet sum source outside planes 0-1";
                }
                uint64_t &w = L.kcoef[src];
                if ((w >> (2 * qq)) & 3u) {
                    code = FLBM_EINVAL;
                    return "two inlet pulls read one population";
                }
                w |= (uint64_t)c << (2 * qq);
            }
        }
    }
    return std::string();
}

namespace {

// Regular sources of direction q over the sites [s0, s0 + tile): the range
// of (source - shift * position) over them; false if an entry is of no kind
// the codes know.
bool source_range(const Lattice &L, int q, int64_t s0, int tile, int shift, int64_t &lo, int64_t &hi)
{
    const int64_t npad = L.n_pad;
    const int32_t *row = L.nbr.data() + (q - 1) * npad;
    const int64_t reg = (int64_t)q * npad, bb = (int64_t)d3q19::opp(q) * npad;
    lo = INT64_MAX;
    hi = INT64_MIN;
    for (int p = 0; p < tile; ++p) {
        const int64_t s = s0 + p, e = row[s];
        if (e == L.sentinel || e == bb + s) continue;
        if (e < reg || e >= reg + npad) return false;
        const int64_t v = e - shift * p;
        lo = std::min(lo, v);
        hi = std::max(hi, v);
    }
    if (lo > hi) lo = hi = reg;  // no regular source in this tile
    return true;
}

uint32_t code_of(const Lattice &L, int q, int64_t s, int64_t base, int64_t p, int form)
{
    const int64_t e = L.nbr[(q - 1) * L.n_pad + s];
    const bool bounce = e == (int64_t)d3q19::opp(q) * L.n_pad + s;
    if (form == PULL_TILE_BYTE)
        return e == L.sentinel ? PULL_BYTE_UNKNOWN : bounce ? PULL_BYTE_BOUNCE : (uint32_t)(e - base - p);
    return e == L.sentinel ? PULL_UNKNOWN : bounce ? PULL_BOUNCE : (uint32_t)(e - base);
}

uint32_t byte_code(const CompactPull &cp, int q, int64_t s, int64_t npad)
{
    return q <= 16 ? (cp.bytes[(size_t)((q - 1) >> 2) * npad + s] >> (((q - 1) & 3) * 8)) & 0xFFu
                   : ((uint32_t)cp.tail[s] >> ((q - 17) * 8)) & 0xFFu;
}

// Run codes of the byte tile starting at s0 (see pull_format.h); false, with
// nothing written, if a wave would list more than PULL_RUN_MAX codes.
bool build_runs(CompactPull &cp, int64_t s0, int tile, int64_t npad, int64_t &wide)
{
    std::vector<uint8_t> list(PULL_RUN_MAX);
    std::vector<uint32_t> mask(PULL_RUN_WAVE), lo(PULL_RUN_WAVE), hi(PULL_RUN_WAVE);
    std::vector<uint32_t> out_lo((size_t)tile * 2), out_hi((size_t)tile);
    int64_t nwide = 0;
    for (int w = 0; w < tile / PULL_RUN_WAVE; ++w) {
        const int64_t sw = s0 + (int64_t)w * PULL_RUN_WAVE;
        std::fill(mask.begin(), mask.end(), 0u);
        int e = 0;
        for (int q = 1; q < 19; ++q)
            for (int l = 0; l < PULL_RUN_WAVE; ++l) {
                const uint32_t c = byte_code(cp, q, sw + l, npad);
                if (l > 0 && c == byte_code(cp, q, sw + l - 1, npad)) continue;
                if (e == PULL_RUN_MAX) return false;
                mask[l] |= 1u << (q - 1);
                list[e++] = (uint8_t)c;
            }
        std::fill(list.begin() + e, list.end(), (uint8_t)0);
        const bool wide_w = e > 4 * PULL_RUN_WAVE;
        nwide += wide_w;
        for (int l = 0; l < PULL_RUN_WAVE; ++l) {
            uint32_t b0 = 0, b1 = 0;
            for (int j = 0; j < 4; ++j) {
                b0 |= (uint32_t)list[4 * l + j] << (8 * j);
                b1 |= (uint32_t)list[4 * PULL_RUN_WAVE + 4 * l + j] << (8 * j);
            }
            const size_t i = (size_t)w * PULL_RUN_WAVE + l;
            out_lo[2 * i] = mask[l] | (wide_w ? PULL_RUN_WIDE : 0u);
            out_lo[2 * i + 1] = b0;
            out_hi[i] = b1;
        }
    }
    std::copy(out_lo.begin(), out_lo.end(), cp.runs.begin() + 2 * s0);
    std::copy(out_hi.begin(), out_hi.end(), cp.runs_hi.begin() + s0);
    wide = nwide;
    return true;
}

}  // namespace

std::string build_compact_pull(const Lattice &L, int tile, int32_t limit16, int32_t limit8, CompactPull &cp)
{
    const int64_t npad = L.n_pad;
    if (tile <= 0 || npad % tile != 0) return "tile does not divide the padded site count";
    if (limit16 < 1 || (uint32_t)limit16 > PULL_MAX_CODE) return "16-bit code limit out of range";
    if (limit8 < 0 || (uint32_t)limit8 > PULL_MAX_BYTE) return "byte code limit out of range";
    cp.tile = tile;
    cp.limit16 = limit16;
    cp.limit8 = limit8;
    cp.tiles = npad / tile;
    try {
        cp.codes.assign((size_t)9 * npad, 0u);
        cp.bytes.assign((size_t)4 * npad, 0u);
        cp.tail.assign((size_t)npad, 0);
        cp.runs.assign((size_t)2 * npad, 0u);
        cp.runs_hi.assign((size_t)npad, 0u);
        cp.hdr.assign((size_t)cp.tiles * PULL_HDR, 0);
    } catch (const std::bad_alloc &) {
        return "host allocation failed while building the compact pull table";
    }
    parallel_for(0, cp.tiles, [&](int64_t t0, int64_t t1) {
        for (int64_t t = t0; t < t1; ++t) {
            const int64_t s0 = t * tile;
            int32_t *h = cp.hdr.data() + t * PULL_HDR;
            int64_t base[19];
            int form = limit8 > 0 ? PULL_TILE_BYTE : PULL_TILE_HALF;
            for (; form > PULL_TILE_INT32; --form) {
                const int shift = form == PULL_TILE_BYTE ? 1 : 0;
                const int64_t lim = form == PULL_TILE_BYTE ? limit8 : limit16;
                bool fits = true;
                for (int q = 1; q < 19 && fits; ++q) {
                    int64_t lo, hi;
                    fits = source_range(L, q, s0, tile, shift, lo, hi) && hi - lo <= lim;
                    base[q] = lo;
                }
                if (fits) break;
            }
            h[PULL_HDR_FORM] = form;
            if (form == PULL_TILE_INT32) continue;
            for (int q = 1; q < 19; ++q) {
                h[q - 1] = (int32_t)base[q];
                for (int64_t p = 0; p < tile; ++p) {
                    const int64_t s = s0 + p;
                    const uint32_t c = code_of(L, q, s, base[q], p, form);
                    if (form == PULL_TILE_HALF) {
                        cp.codes[(size_t)((q - 1) >> 1) * npad + s] |= c << (((q - 1) & 1) * 16);
                    } else if (q <= 16) {
                        cp.bytes[(size_t)((q - 1) >> 2) * npad + s] |= c << (((q - 1) & 3) * 8);
                    } else {
                        cp.tail[s] = (uint16_t)(cp.tail[s] | (c << ((q - 17) * 8)));
                    }
                }
            }
            int64_t wide = 0;
            if (form == PULL_TILE_BYTE && tile % PULL_RUN_WAVE == 0 && build_runs(cp, s0, tile, npad, wide))
                h[PULL_HDR_RUNS] = 1 + (int32_t)wide;  // reduced to the flag below
        }
    });
    cp.tiles16 = cp.tiles8 = cp.tiles_run = cp.waves_wide = 0;
    for (int64_t t = 0; t < cp.tiles; ++t) {
        int32_t *h = cp.hdr.data() + t * PULL_HDR;
        const int f = h[PULL_HDR_FORM];
        cp.tiles16 += f == PULL_TILE_HALF;
        cp.tiles8 += f == PULL_TILE_BYTE;
        if (h[PULL_HDR_RUNS]) {
            cp.tiles_run += 1;
            cp.waves_wide += h[PULL_HDR_RUNS] - 1;
            h[PULL_HDR_RUNS] = 1;
        }
    }
    return std::string();
}

std::string check_compact_pull(const Lattice &L, const CompactPull &cp)
{
    const int64_t npad = L.n_pad;
    if (cp.tile <= 0 || cp.tiles * cp.tile != npad) return "compact table of another lattice";
    for (int64_t t = 0; t < cp.tiles; ++t) {
        const int32_t *h = cp.hdr.data() + t * PULL_HDR;
        const int form = h[PULL_HDR_FORM];
        if (form < PULL_TILE_INT32 || form > PULL_TILE_BYTE || h[PULL_HDR_RUNS] < 0 || h[PULL_HDR_RUNS] > 1 ||
            (h[PULL_HDR_RUNS] && form != PULL_TILE_BYTE))
            return "bad compact tile header";
        if (h[PULL_HDR_RUNS]) {
            // decode the run codes as the step kernel does, lane by lane
            for (int64_t sw = t * cp.tile; sw < (t + 1) * cp.tile; sw += PULL_RUN_WAVE) {
                const bool wide = (cp.runs[(size_t)2 * sw] & PULL_RUN_WIDE) != 0;
                int64_t off = 0;
                for (int q = 1; q < 19; ++q) {
                    int64_t below = 0;
                    for (int l = 0; l < PULL_RUN_WAVE; ++l) {
                        const uint32_t m = cp.runs[(size_t)2 * (sw + l)];
                        if (((m & PULL_RUN_WIDE) != 0) != wide || (m & ~PULL_RUN_WIDE) >> 18) return "bad run mask";
                        const int64_t e = (m >> (q - 1)) & 1u;
                        if (l == 0 && !e) return "run codes without a wave start";
                        const int64_t k = off + below + e - 1;
                        below += e;
                        if (k >= (wide ? 2 : 1) * 4 * PULL_RUN_WAVE) return "run list too long";
                        const uint32_t word = k < 4 * PULL_RUN_WAVE ? cp.runs[(size_t)2 * (sw + k / 4) + 1]
                                                                   : cp.runs_hi[(size_t)(sw + (k - 4 * PULL_RUN_WAVE) / 4)];
                        if (((word >> (8 * (k & 3))) & 0xFFu) != byte_code(cp, q, sw + l, npad))
                            return "run code decodes wrongly";
                    }
                    off += below;
                }
            }
        } else {
            for (int64_t s = t * cp.tile; s < (t + 1) * cp.tile; ++s)
                if (cp.runs[(size_t)2 * s] || cp.runs[(size_t)2 * s + 1] || cp.runs_hi[(size_t)s])
                    return "run codes in a tile without the run flag";
        }
        for (int64_t p = 0; p < cp.tile; ++p) {
            const int64_t s = t * cp.tile + p;
            bool zero16 = true, zero8 = cp.tail[s] == 0;
            for (int k = 0; k < 9; ++k) zero16 &= cp.codes[(size_t)k * npad + s] == 0;
            for (int k = 0; k < 4; ++k) zero8 &= cp.bytes[(size_t)k * npad + s] == 0;
            if ((form != PULL_TILE_HALF && !zero16) || (form != PULL_TILE_BYTE && !zero8))
                return "codes outside the tile's form";
            if (form == PULL_TILE_INT32) continue;
            for (int q = 1; q < 19; ++q) {
                int64_t e;
                if (form == PULL_TILE_HALF) {
                    const uint32_t c = (cp.codes[(size_t)((q - 1) >> 1) * npad + s] >> (((q - 1) & 1) * 16)) & 0xFFFFu;
                    e = c == PULL_UNKNOWN ? L.sentinel
                        : c == PULL_BOUNCE ? (int64_t)d3q19::opp(q) * npad + s
                                           : (int64_t)h[q - 1] + c;
                } else {
                    const uint32_t c = q <= 16 ? (cp.bytes[(size_t)((q - 1) >> 2) * npad + s] >> (((q - 1) & 3) * 8)) & 0xFFu
                                               : ((uint32_t)cp.tail[s] >> ((q - 17) * 8)) & 0xFFu;
                    e = c == PULL_BYTE_UNKNOWN ? L.sentinel
                        : c == PULL_BYTE_BOUNCE ? (int64_t)d3q19::opp(q) * npad + s
                                                : (int64_t)h[q - 1] + p + c;
                }
                if (e != L.nbr[(size_t)(q - 1) * npad + s]) return "compact pull code decodes wrongly";
            }
        }
    }
    return std::string();
}

std::string check_pull_bijection(const Lattice &L, const LatticeSpec &spec)
{
    const int64_t n = L.n, npad = L.n_pad;
    std::vector<uint8_t> seen((size_t)19 * n, 0);
    for (int64_t s = 0; s < n; ++s) seen[s] = 1;  // q = 0 reads its own slot
    for (int q = 1; q < 19; ++q)
        for (int64_t s = 0; s < n; ++s) {
            int64_t idx = L.nbr[(q - 1) * npad + s];
            if (idx == L.sentinel) {
                bool ok = spec.z_mode == FLBM_Z_FLUX &&
                          ((L.coords[3 * s + 2] == 0 && d3q19::cz[q] == 1) ||
                           (L.coords[3 * s + 2] == spec.nz - 1 && d3q19::cz[q] == -1));
                if (!ok) return "sentinel outside a boundary unknown";
                continue;
            }
            int64_t qq = idx / npad, ss = idx % npad;
            if (qq < 0 || qq >= 19 || ss >= n) return "pull index out of range";
            uint8_t &m = seen[qq * n + ss];
            if (m) return "two pulls read one slot";
            m = 1;
        }
    for (int q = 0; q < 19; ++q)
        for (int64_t s = 0; s < n; ++s) {
            if (seen[q * n + s]) continue;
            int z = L.coords[3 * s + 2];
            bool leaves = spec.z_mode == FLBM_Z_FLUX &&
                          ((z == 0 && d3q19::cz[q] == -1) || (z == spec.nz - 1 && d3q19::cz[q] == 1));
            if (!leaves) return "a population is never read";
        }
    return std::string();
}

}  // namespace flbm
