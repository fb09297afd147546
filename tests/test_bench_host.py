"""bench.py's host-side accounting (no GPU): the byte models its roofline
figures use, and its refusal of more than one GPU."""
import subprocess
import sys
from pathlib import Path

import bench

ROOT = Path(__file__).resolve().parents[1]


def test_whole_subcycle_bytes_per_cell():
    # two-pass: 36 nb p + 2 (52 g + 48) + 104; compulsory: 8 nb p + (52 g + 48) + 104
    assert bench.subcycle_bytes_per_cell(3, 4, 4) == {"two_pass": 1048, "compulsory": 456}
    assert bench.subcycle_bytes_per_cell(3, 8, 8) == {"two_pass": 1896, "compulsory": 760}
    assert bench.subcycle_bytes_per_cell(1, 8, 8) == {"two_pass": 1320, "compulsory": 632}


def test_kernel_bytes_per_lattice_cell():
    """Per cell of a six-face lattice (3 faces, 6 face sides), 3 bins, FP32."""
    per_cell = {k: bench.algorithmic_bytes(k, 1, 3, 3, 6, 0, 4, 4)
                for k in ("k_facestate", "k_flux", "k_transport", "k_chem")}
    assert per_cell == {"k_facestate": 548, "k_flux": 616, "k_transport": 344, "k_chem": 200}
    # linear in the cell count
    assert bench.algorithmic_bytes("k_flux", 1000, 3, 3000, 6000, 0, 4, 4) == 616 * 1000


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
