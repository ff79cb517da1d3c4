"""CPU checks of bench.py's host logic: one GPU only, and the kernel-name
parsing that maps rocprofv3 trace rows to sweep kinds (trace names of kernels
with _Float16 arguments stay mangled)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, cwd=ROOT, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)


def test_kernel_names_map_to_sweep_kinds():
    import bench
    cases = {
        "void hlbm::k_primal<19, float, true, 3, false>(hlbm::Geo, hlbm::Coll)": ("primal_window", "true"),
        "void hlbm::k_primal_stream<9, double, false, 0, false>(hlbm::Geo)": ("primal", "false"),
        "_ZN4hlbm8k_primalILi19EDF16_Lb1ELi0ELb0EEEvNS_3GeoENS_4CollE": ("primal", "true"),
        "_ZN4hlbm15k_primal_streamILi9EDF16_Lb0ELi3ELb1EEEvNS_3GeoE": ("primal_window", "false"),
        "void hlbm::k_primal_wstream<19, float, true, 3, false>(hlbm::Geo)": ("primal_window", "true"),
        "void hlbm::k_adjoint<19, float, true, false, false>(hlbm::Geo)": ("adjoint", "true"),
        "void hlbm::k_adjoint_stream<9, double, false, false>(hlbm::Geo)": ("adjoint", "false"),
        "void hlbm::k_adjoint_pstream<19, float, false, false>(hlbm::Geo)": ("adjoint", "true"),
        "void hlbm::k_window_region<19, float, false>(hlbm::Geo)": ("region", None),
        "void hlbm::k_window_region_copy<19, float>(hlbm::ObjBox, float const*, double*)": ("region", None),
        "_ZN4hlbm20k_window_region_copyILi9EdEEvNS_6ObjBoxEPKT0_Pd": ("region", None),
        "_ZN4hlbm12k_copy_probeILi19EDF16_Lb1ELb1EEEvNS_3GeoE": ("copy_odd_nt", None),
        "void hlbm::k_copy_probe<9, float, false, false>(hlbm::Geo)": ("copy_own", None),
        "void hlbm::k_copy_probe_pull<19, float>(hlbm::Geo, float const*, float*)": ("copy_pull", None),
        "void hlbm::k_gradient<9, double, double>(hlbm::Geo)": (None, None),
        "__amd_rocclr_copyBuffer": (None, None),
    }
    for name, want in cases.items():
        assert bench.kernel_kind(name) == want, name
    assert bench._itanium_kernel("_ZN4hlbm8k_primalILi19EDF16_Lb1ELi0ELb0EEEvNS_3GeoE") == \
        ("k_primal", ["19", "_Float16", "true", "0", "false"])
