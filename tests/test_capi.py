"""CPU checks of the C ABI: the library loads without a GPU and exports every
function include/hlbm.h declares, with matching struct sizes."""
import ctypes as C
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hlbm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hlbm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for must in ["hlbm_create", "hlbm_destroy", "hlbm_set_porosity", "hlbm_build_cylinder",
                 "hlbm_set_objective", "hlbm_run_primal", "hlbm_solve_adjoint",
                 "hlbm_get_objective", "hlbm_get_gradient"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    from paper_2606_31707_amd import hlbm as H
    lib = H.load_library()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(H.EXPORTS) == declared_functions()
    out = subprocess.run(["nm", "-D", "--defined-only", H.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (hlbm_[a-z_]+)", out))
    assert set(declared_functions()) <= exported


def test_struct_layouts_match_header():
    """Compiles a tiny C program against the header and compares sizeof/offsets
    with the ctypes mirrors."""
    from paper_2606_31707_amd import hlbm as H
    src = r'''
#include <stdio.h>
#include <stddef.h>
#include "hlbm.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(hlbm_desc), offsetof(hlbm_desc, force),
         offsetof(hlbm_desc, stream), sizeof(hlbm_adjoint_opts), offsetof(hlbm_adjoint_opts, restart),
         sizeof(hlbm_adjoint_report));
  return 0;
}
'''
    import tempfile
    with tempfile.TemporaryDirectory() as td:
        cpath = os.path.join(td, "t.c")
        open(cpath, "w").write(src)
        exe = os.path.join(td, "t")
        subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), cpath, "-o", exe], check=True)
        vals = list(map(int, subprocess.run([exe], capture_output=True, text=True).stdout.split()))
    assert vals == [C.sizeof(H.Desc), H.Desc.force.offset, H.Desc.stream.offset, C.sizeof(H.AdjointOpts),
                    H.AdjointOpts.restart.offset, C.sizeof(H.AdjointReport)]


def test_status_strings_without_gpu():
    from paper_2606_31707_amd import hlbm as H
    lib = H.load_library()
    assert lib.hlbm_status_string(H.E_STATE) == b"call order violated"
    d = H.make_desc(nx=1, ny=1)
    with pytest.raises(H.HlbmError):
        H.footprint_bytes(d)
    d = H.make_desc(nx=220, ny=41)
    assert H.footprint_bytes(d, False, False) >= 220 * 41 * (9 * 8 + 8)
    for policy in (H.CACHE_AUTO, H.CACHE_PLAIN, H.CACHE_STREAMING):
        assert H.footprint_bytes(H.make_desc(nx=220, ny=41, cache_policy=policy), False, False) > 0
    for policy in (-1, 3):
        with pytest.raises(H.HlbmError):
            H.footprint_bytes(H.make_desc(nx=220, ny=41, cache_policy=policy))


def test_product_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2606_31707_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, f)).read()
                assert not re.search(r"^\s*(from|import)\s+oracle", text, flags=re.M), f
                assert "hlbm_oracle" not in text, f


def test_footprint_counts_the_objective_region_without_gpu():
    from paper_2606_31707_amd import hlbm as H
    d = H.make_desc(nx=220, ny=41)
    base = H.footprint_bytes(d, True, True)
    diss = H.footprint_bytes(d, True, True, 200 * 41, H.OBJ_DISS)
    mea = H.footprint_bytes(d, True, True, 200 * 41, H.OBJ_MEA)
    rp = -(-200 * 41 // 128) * 128
    assert diss - base == 2 * 8 * 8 * rp          # two arrays of 8 FP64 coefficients per region cell
    assert mea - diss == rp + 8 * 9 * rp           # surface flags and the constant source
    for bad in [(-1, H.OBJ_DISS), (220 * 41 + 1, H.OBJ_DISS), (10, 7)]:
        with pytest.raises(H.HlbmError):
            H.footprint_bytes(d, True, True, *bad)


def test_footprint_counts_pending_window_values_and_the_region_record_without_gpu():
    """The grouped window accumulation holds three FP32 pending slots of
    (2 + dim [+ q]) planes on FP32/FP16 lattices (none in FP64); a drag plane
    (a moment-form region of at most 1/8 of the lattice) holds one record of
    whole 128-byte lines per region cell for the region pass."""
    from paper_2606_31707_amd import hlbm as H
    from paper_2606_31707_amd import inputs as I
    w = I.les_re3900()
    for prec, track in ((H.FP64, False), (H.FP32, False), (H.FP16S, False), (H.FP32, True)):
        d = H.make_desc(stencil=H.D3Q19, precision=prec, nx=w.nx, ny=w.ny, nz=w.nz, tau=w.tau, cs=w.cs,
                        bc_x=H.BC_INLET_OUTLET, bc_y=w.bc_y, bc_z=w.bc_z, inlet_profile=w.inlet_profile,
                        u_in=w.u_max, track_mean_populations=track)
        ssize = {H.FP64: 8, H.FP32: 4, H.FP16S: 2}[prec]
        unit = 256 // ssize
        m = -(-w.n // unit)
        plane = (m + 1 if m % 2 == 0 else m) * unit  # odd number of 256-byte blocks
        sums = plane * 8 * (1 + 3 + 1 + (19 if track else 0))
        pending = 0 if prec == H.FP64 else 3 * plane * 4 * (2 + 3 + (19 if track else 0))
        assert H.footprint_bytes(d, True, False) - H.footprint_bytes(d, False, False) == sums + pending
        cells = 288 * 128  # the drag plane x = 432, y 48..335
        rp = -(-cells // 128) * 128
        asz = 8 if prec == H.FP64 else 4
        record = -(-20 // (128 // asz)) * (128 // asz)  # 19 populations and d, padded to 128-byte lines
        ffa = H.footprint_bytes(d, True, False, cells, H.OBJ_FFA) - H.footprint_bytes(d, True, False)
        assert ffa == 2 * 8 * 12 * rp + rp * record * asz
        big = w.n // 8 + 1  # above 1/8 of the lattice the terms are fused into the sweep: no record
        rbig = -(-big // 128) * 128
        assert H.footprint_bytes(d, True, False, big, H.OBJ_DISS) - H.footprint_bytes(d, True, False) == \
            2 * 8 * 12 * rbig
