"""CPU checks of bench.py's reporting contract: the committed rocprofv3
summary of the pass kernel was taken on the committed kernel source (so the
bench's `roofline.traffic` is not null), its traffic figure is consistent
with the algorithmic bytes of one launch, and more than one GPU is refused."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_profile_matches_kernel_source():
    t = bench.measured_traffic()
    assert t is not None, "profiles/sv_pass_kernel_1080p.md was taken on another filter.hip: retake it"
    # per launch of the default step: the algorithmic bytes of 32 frames; the
    # measured HBM traffic lies between them and twice them
    alg = bench.PASS_BYTES_PER_PX * bench.H * bench.W * 32
    assert alg <= t <= 2 * alg


def test_comment_edits_keep_the_hash(tmp_path):
    src = os.path.join(ROOT, "paper_2512_04556_amd", "csrc", "filter.hip")
    text = open(src).read()
    edited = tmp_path / "f.hip"
    edited.write_text("// a new comment\n\n" + text.replace("\n", "  // trailing\n", 3))
    assert bench.source_code_bytes(str(edited)) == bench.source_code_bytes(src)
    changed = tmp_path / "g.hip"
    changed.write_text(text + "\nint extra_symbol;\n")
    assert bench.source_code_bytes(str(changed)) != bench.source_code_bytes(src)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
