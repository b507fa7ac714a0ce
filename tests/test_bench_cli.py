"""Host-side pieces of the measurement (CPU): the one-GPU guard of bench.py,
its algorithmic byte model, and the traffic record that bench.py reports
only for the kernel build it was measured on."""
import json
import os
import subprocess
import sys

from paper_0901_4107_amd.build import source_hash
from paper_0901_4107_amd.prof_summary import read_traffic

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_flux_byte_model():
    sys.path.insert(0, ROOT)
    import bench
    # per face: L, R; A, g, d in the path's precision; w_f and the 5 fluxes
    # in double. Per cell: W, its gradient and s - r in the path's precision.
    nbytes, pf, pc = bench.flux_kernel_bytes(3, 10, 100, mixed=False)
    assert (pf, pc) == (8 + 7 * 8 + 3 * 8 + 5 * 8, 23 * 8)
    nbytes_m, pfm, pcm = bench.flux_kernel_bytes(3, 10, 100, mixed=True)
    assert (pfm, pcm) == (8 + 7 * 4 + 3 * 8 + 5 * 8, 23 * 4)
    # the headline mesh: 100 B per face and 92 B per cell in the mixed form
    assert bench.flux_kernel_bytes(3, 2097152, 16291535, mixed=True)[0] == 16291535 * 100 + 2097152 * 92
    assert nbytes == 100 * pf + 10 * pc and nbytes_m == 100 * pfm + 10 * pcm


def test_traffic_record_follows_the_kernel_sources(tmp_path):
    good = (f"traffic: kernel=k_face_flux_mixed<3, true, false, false> workload=w read_bytes=100 written_bytes=20 "
            f"source={source_hash()}\n")
    stale = "traffic: kernel=k_face_flux64<3, false, false, false> workload=w read_bytes=7 written_bytes=1 source=0000000000000000\n"
    (tmp_path / "t.md").write_text("# summary\n\n" + good + stale)
    assert read_traffic(str(tmp_path), "k_face_flux_mixed<3, true, false, false>", "w") == 120.0
    assert read_traffic(str(tmp_path), "k_face_flux64<3, false, false, false>", "w") is None    # other sources
    assert read_traffic(str(tmp_path), "k_face_flux_mixed<3, true, false, false>", "other") is None
