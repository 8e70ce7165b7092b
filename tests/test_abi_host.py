"""CPU-side tests of the C-ABI library: it loads, exports every declared
symbol, and its host logic (parameter checks, sparse lattice and pull table)
agrees with a brute-force derivation. No compute call is made."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1806_10589_amd import fluxlbm, inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fluxlbm.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(flbm_[a-z0-9_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = fluxlbm.load_library()
    names = _declared()
    assert len(names) > 20
    for name in names:
        assert hasattr(lib, name), name
    # and the binding wraps exactly those names
    assert set(fluxlbm.exported_symbols()) == set(names)


def test_params_struct_layout():
    # 10 int32 then 8 doubles, no padding
    assert ctypes.sizeof(fluxlbm.flbm_params) == 10 * 4 + 8 * 8
    p = fluxlbm.flbm_default_params()
    assert p.tau == 0.8 and p.rho0 == 1.0 and p.umax_limit == 0.1
    assert p.precision == fluxlbm.FLBM_FP32 and p.z_mode == fluxlbm.FLBM_Z_FLUX


def test_struct_layouts_match_the_header(tmp_path):
    # compile the header with the host C compiler and compare every field
    # offset and the struct sizes with the ctypes mirrors
    structs = {"flbm_params": fluxlbm.flbm_params,
               "flbm_controller_params": fluxlbm.flbm_controller_params,
               "flbm_schedule": fluxlbm.flbm_schedule}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "fluxlbm.h"', "int main(void){"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} %zu\\n", sizeof({name}));')
        for fname, _ in cls._fields_:
            lines.append(f'printf("{name}.{fname} %zu\\n", offsetof({name}, {fname}));')
    lines.append("return 0;}")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    import subprocess
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = dict(l.split() for l in subprocess.run([str(exe)], capture_output=True, text=True,
                                                  check=True).stdout.splitlines())
    for name, cls in structs.items():
        assert int(out[name]) == ctypes.sizeof(cls), name
        for fname, _ in cls._fields_:
            assert int(out[f"{name}.{fname}"]) == getattr(cls, fname).offset, (name, fname)


def test_mlp_parameter_count():
    # 32 -> 128 -> 128 -> 1 with biases
    assert fluxlbm.flbm_mlp_num_params() == 128 * 32 + 128 + 128 * 128 + 128 + 128 + 1


def _params(mask, **kw):
    p = fluxlbm.flbm_default_params()
    p.nz, p.ny, p.nx = mask.shape
    for k, v in kw.items():
        setattr(p, k, v)
    return p


def test_invalid_parameters_rejected():
    mask = np.zeros((5, 4, 4), np.uint8)
    for kw in ({"tau": 0.5}, {"rho0": 0.0}, {"z_mode": 7}, {"precision": 9},
               {"reservoir_layers": 3}, {"watchdog_every": -1}):
        with pytest.raises(fluxlbm.FlbmError) as e:
            fluxlbm.flbm_create(mask, _params(mask, **kw))
        assert e.value.status == fluxlbm.FLBM_EINVAL
    small = np.zeros((2, 4, 4), np.uint8)
    with pytest.raises(fluxlbm.FlbmError):
        fluxlbm.flbm_create(small, _params(small))


def test_all_solid_inlet_is_enoinlet():
    mask = np.zeros((6, 4, 4), np.uint8)
    mask[0] = 1
    with pytest.raises(fluxlbm.FlbmError) as e:
        fluxlbm.flbm_create(mask, _params(mask))
    assert e.value.status == fluxlbm.FLBM_ENOINLET
    # reservoirs clear the inlet plane again
    ctx = fluxlbm.flbm_create(mask, _params(mask, reservoir_layers=1))
    assert fluxlbm.flbm_num_sites(ctx)[1] == 16
    fluxlbm.flbm_destroy(ctx)


def test_mask_without_pores_is_einval():
    mask = np.ones((6, 4, 4), np.uint8)
    for z_mode in (fluxlbm.FLBM_Z_FLUX, fluxlbm.FLBM_Z_PERIODIC):
        with pytest.raises(fluxlbm.FlbmError) as e:
            fluxlbm.flbm_create(mask, _params(mask, z_mode=z_mode))
        assert e.value.status == fluxlbm.FLBM_EINVAL


def test_lattice_beyond_32_bit_indices_is_eindex():
    # The largest flat index is 19 n_pad plus the 64-element pad behind the
    # sentinel; n_pad (a multiple of 1024) may reach 113,025,024. One pore
    # site more pads to 113,026,048 and is refused, before any per-site
    # allocation.
    mask = np.zeros((484, 484, 484), np.uint8)
    flat = mask.reshape(-1)
    plane = 484 * 484
    flat[plane:plane + mask.size - 113_025_025] = 1
    with pytest.raises(fluxlbm.FlbmError) as e:
        fluxlbm.flbm_create(mask, _params(mask))
    assert e.value.status == fluxlbm.FLBM_EINDEX


def _brute_pull(mask, px, py, z_mode, npad):
    """Expected pull index of (q, s) from the definition of streaming."""
    cx = [0, 1, -1, 0, 0, 0, 0, 1, -1, 1, -1, 1, -1, 1, -1, 0, 0, 0, 0]
    cy = [0, 0, 0, 1, -1, 0, 0, 1, -1, -1, 1, 0, 0, 0, 0, 1, -1, 1, -1]
    cz = [0, 0, 0, 0, 0, 1, -1, 0, 0, 0, 0, 1, -1, -1, 1, 1, -1, -1, 1]
    opp = [0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17]
    nz, ny, nx = mask.shape
    sites = inputs.pore_sites(mask)
    index = {int(c): s for s, c in enumerate(sites)}
    out = np.zeros((18, len(sites)), np.int64)
    for s, c in enumerate(sites):
        z, rem = divmod(int(c), ny * nx)
        y, x = divmod(rem, nx)
        for q in range(1, 19):
            sx, sy, sz = x - cx[q], y - cy[q], z - cz[q]
            if not 0 <= sz < nz:
                if z_mode == 0:
                    out[q - 1, s] = 19 * npad
                    continue
                if z_mode == 1:
                    sz %= nz
                else:
                    out[q - 1, s] = opp[q] * npad + s
                    continue
            wall = False
            if not 0 <= sx < nx:
                if px:
                    sx %= nx
                else:
                    wall = True
            if not 0 <= sy < ny:
                if py:
                    sy %= ny
                else:
                    wall = True
            if not wall and mask[sz, sy, sx]:
                wall = True
            if wall:
                out[q - 1, s] = opp[q] * npad + s
            else:
                out[q - 1, s] = q * npad + index[(sz * ny + sy) * nx + sx]
    return out


@pytest.mark.parametrize("z_mode", [0, 1, 2])
@pytest.mark.parametrize("px,py", [(0, 0), (1, 0), (1, 1)])
def test_pull_table_matches_definition(z_mode, px, py):
    mask = inputs.random_mask((7, 5, 6), 0.3, 90 + z_mode)
    mask[0, 0, 0] = 0
    ctx = fluxlbm.flbm_create(mask, _params(mask, periodic_x=px, periodic_y=py, z_mode=z_mode))
    n, a_in, a_out = fluxlbm.flbm_num_sites(ctx)
    assert n == int((mask == 0).sum())
    assert a_in == int((mask[0] == 0).sum()) and a_out == int((mask[-1] == 0).sum())
    coords = fluxlbm.flbm_get_site_coords(ctx, n)
    sites = inputs.pore_sites(mask)
    nz, ny, nx = mask.shape
    assert np.array_equal(coords[:, 0] + nx * (coords[:, 1] + ny * coords[:, 2]), sites)
    nbr = fluxlbm.flbm_get_pull_table(ctx, n)
    _, _, npad = fluxlbm.flbm_device_layout(ctx)
    assert npad % 1024 == 0 and npad >= n
    assert np.array_equal(nbr, _brute_pull(mask, px, py, z_mode, npad))
    fluxlbm.flbm_destroy(ctx)


def test_sphere_pack_generator_is_seeded_and_hits_porosity():
    m1, phi1, k1 = inputs.sphere_pack(48, 0.35, seed=2, reservoir_layers=6)
    m2, phi2, k2 = inputs.sphere_pack(48, 0.35, seed=2, reservoir_layers=6)
    assert np.array_equal(m1, m2) and phi1 == phi2 and k1 == k2
    assert 0.33 < phi1 <= 0.35
    assert not m1[:6].any() and not m1[-6:].any()
    m3, _, _ = inputs.sphere_pack(48, 0.35, seed=3)
    assert not np.array_equal(m1, m3)


def test_batch_and_network_argument_checks_without_a_device():
    lib = fluxlbm.load_library()
    out = ctypes.c_void_p()
    assert lib.flbm_batch_create(0, None, ctypes.byref(out)) == fluxlbm.FLBM_EINVAL
    assert lib.flbm_batch_create(2, None, ctypes.byref(out)) == fluxlbm.FLBM_EINVAL
    assert lib.flbm_mlp_create(0, None, ctypes.byref(out)) == fluxlbm.FLBM_EINVAL
    assert lib.flbm_batch_set_schedule(None, None) == fluxlbm.FLBM_EINVAL
    assert lib.flbm_gemm_bf16(None, 1, 1, None, 1, 1, None, 1, 1, 1, 1, None) == fluxlbm.FLBM_EINVAL
    assert lib.flbm_set_controller(None, None, None) == fluxlbm.FLBM_EINVAL
    assert lib.flbm_pull_run_info(None, None, None) == fluxlbm.FLBM_EINVAL
    assert lib.flbm_get_pull_runs(None, None, None) == fluxlbm.FLBM_EINVAL


_OPP = [0, 2, 1, 4, 3, 6, 5, 8, 7, 10, 9, 12, 11, 14, 13, 16, 15, 18, 17]


def _decode_compact(codes16, codes8, tail, hdr, npad, n):
    """Flat pull indices [18][n] that the coded tiles give, and each site's
    tile form (0: int32 table, 1: 16-bit codes, 2: 8-bit codes)."""
    tile = npad // hdr.shape[0]
    s = np.arange(n)
    t = s // tile
    p = s % tile
    form = hdr[t, 18]
    out = np.full((18, n), -1, np.int64)
    for q in range(1, 19):
        base = hdr[t, q - 1].astype(np.int64)
        c16 = (codes16[(q - 1) // 2, :n].astype(np.int64) >> (16 * ((q - 1) % 2))) & 0xFFFF
        d16 = np.where(c16 == 0xFFFE, 19 * npad, np.where(c16 == 0xFFFF, _OPP[q] * npad + s, base + c16))
        if q <= 16:
            c8 = (codes8[(q - 1) // 4, :n].astype(np.int64) >> (8 * ((q - 1) % 4))) & 0xFF
        else:
            c8 = (tail[:n].astype(np.int64) >> (8 * (q - 17))) & 0xFF
        d8 = np.where(c8 == 0xFE, 19 * npad, np.where(c8 == 0xFF, _OPP[q] * npad + s, base + p + c8))
        out[q - 1] = np.where(form == 1, d16, np.where(form == 2, d8, -1))
    return out, form


def _compact(ctx):
    n, _, _ = fluxlbm.flbm_num_sites(ctx)
    _, _, npad = fluxlbm.flbm_device_layout(ctx)
    fmt, t8, t16, tiles = fluxlbm.flbm_pull_format_info(ctx)
    codes16, codes8, tail, hdr = fluxlbm.flbm_get_compact_pull(ctx, npad, tiles)
    got, form = _decode_compact(codes16, codes8, tail, hdr, npad, n)
    return n, npad, (fmt, t8, t16, tiles), got, form, (codes16, codes8, tail, hdr)


@pytest.mark.parametrize("z_mode", [0, 1, 2])
@pytest.mark.parametrize("px,py", [(0, 0), (1, 1)])
@pytest.mark.parametrize("fmt", [1, 2])
def test_compact_pull_table_decodes_to_the_definition(z_mode, px, py, fmt):
    mask = inputs.random_mask((9, 23, 17), 0.3, 40 + z_mode)
    mask[0, 0, 0] = 0
    ctx = fluxlbm.flbm_create(mask, _params(mask, periodic_x=px, periodic_y=py, z_mode=z_mode))
    try:
        assert fluxlbm.flbm_pull_format_info(ctx)[0] == fluxlbm.FLBM_PULL_RUN  # the default
        fluxlbm.flbm_set_pull_format(ctx, fmt)
        n, npad, info, got, form, (_, _, _, hdr) = _compact(ctx)
        assert info[0] == fmt and info[3] == npad // 512
        assert info[1] + info[2] == info[3]          # no tile of this small box needs int32
        if fmt == fluxlbm.FLBM_PULL_HALF:
            assert info[1] == 0
        assert np.array_equal(got, _brute_pull(mask, px, py, z_mode, npad))
        assert set(np.unique(hdr[:, 19])) <= {0, 1} and not hdr[hdr[:, 18] != 2, 19].any()
    finally:
        fluxlbm.flbm_destroy(ctx)


def test_compact_pull_table_falls_back_per_tile():
    # a 48^3 pack with reservoirs; small code limits send the tiles whose
    # sources spread wider (a y-wrap, sources a plane apart) to wider forms
    mask, _, _ = inputs.sphere_pack(48, 0.35, seed=7, reservoir_layers=4)
    ctx = fluxlbm.flbm_create(mask, _params(mask))
    try:
        n, npad, info, _, _, _ = _compact(ctx)
        nbr = fluxlbm.flbm_get_pull_table(ctx, n).astype(np.int64)
        tiles = info[3]
        assert 0 < info[1] < tiles and info[1] + info[2] == tiles  # byte and 16-bit tiles, no int32
        fluxlbm.flbm_set_pull_format(ctx, fluxlbm.FLBM_PULL_COMPACT, 600, 100)
        n, npad, info, got, form, (c16, c8, tail, hdr) = _compact(ctx)
        assert info[1] > 0 and info[2] > 0 and info[1] + info[2] < tiles   # all three forms
        coded = form > 0
        assert np.array_equal(got[:, coded], nbr[:, coded])
        # rows of the forms a tile does not use are zero, and int32 tiles have no header
        t_form = hdr[:, 18]
        assert not hdr[t_form == 0].any()
        assert not c16.reshape(9, tiles, 512)[:, t_form != 1].any()
        assert not c8.reshape(4, tiles, 512)[:, t_form != 2].any()
        assert not tail.reshape(tiles, 512)[t_form != 2].any()
        assert not hdr[t_form != 2, 19].any()
        # an int32 tile really spans more than the 16-bit limit in some direction
        t = int(np.flatnonzero(t_form == 0)[0])
        rows = nbr[:, t * 512:min(n, (t + 1) * 512)]
        spans = [int(r[(r // npad) == q].max() - r[(r // npad) == q].min()) if ((r // npad) == q).any() else 0
                 for q, r in zip(range(1, 19), rows)]
        assert max(spans) > 600
        # defaults again; 16-bit only; then the int32 table
        fluxlbm.flbm_set_pull_format(ctx, fluxlbm.FLBM_PULL_COMPACT)
        assert fluxlbm.flbm_pull_format_info(ctx)[1:3] == tuple(_compact(ctx)[2][1:3])
        fluxlbm.flbm_set_pull_format(ctx, fluxlbm.FLBM_PULL_HALF)
        assert fluxlbm.flbm_pull_format_info(ctx)[1:3] == (0, tiles)
        fluxlbm.flbm_set_pull_format(ctx, fluxlbm.FLBM_PULL_INT32)
        assert fluxlbm.flbm_pull_format_info(ctx) == (fluxlbm.FLBM_PULL_INT32, 0, 0, tiles)
        for bad in ((7, 0, 0), (2, 0x10000, 0), (2, 0, 0x100), (2, -1, 0)):
            with pytest.raises(fluxlbm.FlbmError):
                fluxlbm.flbm_set_pull_format(ctx, *bad)
    finally:
        fluxlbm.flbm_destroy(ctx)


def _byte_codes(codes8, tail, s, q):
    if q <= 16:
        return (codes8[(q - 1) // 4, s].astype(np.int64) >> (8 * ((q - 1) % 4))) & 0xFF
    return (tail[s].astype(np.int64) >> (8 * (q - 17))) & 0xFF


@pytest.mark.parametrize("case", ["pack", "random"])
def test_run_codes_decode_to_the_byte_codes(case):
    """Run codes (pull_format.h): per wave of 64 sites, the mask of the
    directions whose byte code changes at each site and the list of the
    changed codes. Decoded here with a running count per direction (not the
    lane arithmetic of the kernel), they give every 8-bit code of every tile
    that carries them; the tiles without them are exactly the 8-bit tiles
    with a wave that would list more than 512 codes; the wide flag marks
    exactly the waves listing more than 256."""
    if case == "pack":
        mask, _, _ = inputs.sphere_pack(48, 0.35, seed=7, reservoir_layers=4)
    else:
        mask = inputs.random_mask((20, 40, 40), 0.5, 3)
    ctx = fluxlbm.flbm_create(mask, _params(mask))
    try:
        n, npad, info, _, form, (_, codes8, tail, hdr) = _compact(ctx)
        runs, runs_hi = fluxlbm.flbm_get_pull_runs(ctx, npad)
        n_runs, n_wide = fluxlbm.flbm_pull_run_info(ctx)
        tiles = info[3]
        flag = hdr[:, 19]
        assert set(np.unique(flag)) <= {0, 1} and not flag[hdr[:, 18] != 2].any() and flag.sum() == n_runs
        wide_seen = 0
        for t in range(tiles):
            if hdr[t, 18] != 2:
                assert not runs[t * 512:(t + 1) * 512].any() and not runs_hi[t * 512:(t + 1) * 512].any()
                continue
            longest = 0
            for w in range(8):
                s = np.arange(t * 512 + 64 * w, t * 512 + 64 * w + 64)
                listed = [np.r_[True, _byte_codes(codes8, tail, s, q)[1:] != _byte_codes(codes8, tail, s, q)[:-1]]
                          for q in range(1, 19)]
                e_total = int(sum(x.sum() for x in listed))
                longest = max(longest, e_total)
                if not flag[t]:
                    continue
                m = runs[s, 0]
                wide = (m >> 31) & 1
                assert (wide == (e_total > 256)).all()
                wide_seen += int(e_total > 256)
                lst = np.concatenate([np.ascontiguousarray(runs[s, 1]).view(np.uint8),
                                      np.ascontiguousarray(runs_hi[s]).view(np.uint8)]).astype(np.int64)
                off = 0
                for q in range(1, 19):
                    e = ((m >> (q - 1)) & 1).astype(bool)
                    assert np.array_equal(e, listed[q - 1])
                    got = lst[off + np.cumsum(e) - 1]
                    off += int(e.sum())
                    assert np.array_equal(got, _byte_codes(codes8, tail, s, q))
                assert not (m & 0x7FFC0000).any()
            assert (longest <= 512) == bool(flag[t])
        assert wide_seen == n_wide
        if case == "random":
            assert 0 < n_runs < info[1] and n_wide > 0   # both kinds of 8-bit tile
        else:
            assert n_runs == info[1]
    finally:
        fluxlbm.flbm_destroy(ctx)


def test_colour_model_reads_the_compact_pull_table():
    mask = inputs.random_mask((6, 8, 8), 0.2, 5)
    mask[0] = 0
    ctx = fluxlbm.flbm_create(mask, _params(mask, model=fluxlbm.FLBM_COLOUR))
    try:
        fmt, t8, t16, tiles = fluxlbm.flbm_pull_format_info(ctx)
        assert fmt == fluxlbm.FLBM_PULL_RUN and t8 + t16 <= tiles and tiles >= 1
        for fmt in (fluxlbm.FLBM_PULL_HALF, fluxlbm.FLBM_PULL_INT32, fluxlbm.FLBM_PULL_COMPACT,
                    fluxlbm.FLBM_PULL_RUN):
            fluxlbm.flbm_set_pull_format(ctx, fmt)
            assert fluxlbm.flbm_pull_format_info(ctx)[0] == fmt
    finally:
        fluxlbm.flbm_destroy(ctx)


def test_no_buffer_path_has_no_compact_pull_table(monkeypatch):
    """FLBM_NO_BUF=1 (testing aid) takes the 64-bit addressing path of
    lattices past 4 GiB, which reads the int32 table only."""
    mask = inputs.random_mask((6, 8, 8), 0.2, 5)
    mask[0] = 0
    monkeypatch.setenv("FLBM_NO_BUF", "1")
    ctx = fluxlbm.flbm_create(mask, _params(mask, model=fluxlbm.FLBM_COLOUR))
    try:
        assert fluxlbm.flbm_pull_format_info(ctx)[:3] == (fluxlbm.FLBM_PULL_INT32, 0, 0)
        for fmt in (fluxlbm.FLBM_PULL_HALF, fluxlbm.FLBM_PULL_COMPACT, fluxlbm.FLBM_PULL_RUN):
            with pytest.raises(fluxlbm.FlbmError) as e:
                fluxlbm.flbm_set_pull_format(ctx, fmt)
            assert e.value.status == fluxlbm.FLBM_ESTATE
        assert fluxlbm.flbm_pull_run_info(ctx) == (0, 0)
        with pytest.raises(fluxlbm.FlbmError) as e:
            fluxlbm.flbm_get_pull_runs(ctx, 1024)
        assert e.value.status == fluxlbm.FLBM_ESTATE
    finally:
        fluxlbm.flbm_destroy(ctx)


def test_profiling_switch_on_the_host(monkeypatch):
    """FLBM_PROFILE=1 opens the roctx library lazily; on a host without a GPU
    a step still fails cleanly with a HIP error and no crash."""
    mask = inputs.random_mask((6, 8, 8), 0.2, 5)
    mask[0] = 0
    monkeypatch.setenv("FLBM_PROFILE", "1")
    ctx = fluxlbm.flbm_create(mask, _params(mask))
    try:
        rc = fluxlbm.load_library().flbm_step(ctx, 3)
        assert rc in (fluxlbm.FLBM_OK, fluxlbm.FLBM_EHIP)
    finally:
        fluxlbm.flbm_destroy(ctx)
