"""Resource use of the tile kernels (voxel tiles, the tiled diagonal and the convolution), read from the gfx950 code-object
metadata that hipcc writes for them: no private (scratch) memory, which a
register array indexed at run time or a vector-register spill would silently
bring in (every access then goes through the vector-memory path).  Scalar
registers may spill into lanes of vector registers, which needs no memory."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1804_10541_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _kernel_metadata(src, tmp_path):
    if not os.path.exists(HIPCC) and shutil.which("hipcc") is None:
        pytest.skip("hipcc not available")
    out = tmp_path / (os.path.basename(src) + ".s")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-I" + os.path.join(ROOT, "include"), "--cuda-device-only", "-S",
           os.path.join(CSRC, src), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    text = out.read_text()
    meta = {}
    for blk in re.findall(r"(- \.agpr_count.*?\.wavefront_size:\s+\d+)", text, re.S):
        name = re.search(r"\.name:\s+(\S+)", blk).group(1)
        field = lambda k: int(re.search(r"\." + k + r":\s+(\d+)", blk).group(1))
        meta[name] = {k: field(k) for k in ("private_segment_fixed_size", "vgpr_spill_count", "sgpr_spill_count",
                                            "vgpr_count")}
    return meta


# VGPR bounds: 128 = four waves per SIMD (two 512-thread groups per CU); the
# convolution's 256-thread groups are held to three per CU by their 50 KB of
# LDS, so three waves per SIMD (168 VGPRs) suffice there.
@pytest.mark.parametrize("src,kernel,max_vgpr", [("ngf_tile.hip", "ngf_tile_kernel", 128),
                                                 ("ngf_tile.hip", "ngf_tile_batch_kernel", 128),
                                                 ("plane_tile.hip", "plane_tile_kernel", 128),
                                                 ("diag_tile.hip", "diag_tile_kernel", 128),
                                                 ("cnn_kernels.hip", "cnn_conv_kernel", 168)])
def test_tile_kernels_use_no_scratch_memory(src, kernel, max_vgpr, tmp_path):
    meta = _kernel_metadata(src, tmp_path)
    tiles = {k: v for k, v in meta.items() if kernel in k}
    assert tiles, f"no {kernel} instances in {src}"
    for name, m in tiles.items():
        assert m["private_segment_fixed_size"] == 0, (name, m)
        assert m["vgpr_spill_count"] == 0, (name, m)
        assert m["vgpr_count"] <= max_vgpr, (name, m)
