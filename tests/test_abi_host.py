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
