"""The bench's reading of committed rocprofv3 summaries (CPU only): each
traversal profile is recognised as the BVH4 variant it was taken on, with
or without the kernel's extra integer argument."""
import os

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _kernel_of(name):
    for line in open(os.path.join(ROOT, "profiles", name)):
        if line.startswith("kernel:"):
            return line.split(":", 1)[1].strip()
    raise AssertionError(f"{name} names no kernel")


def test_traversal_profiles_match_their_bvh_width():
    for name in ("trace_hit_boxfield_pmc.txt", "trace_shade_boxfield_pmc.txt"):
        k = _kernel_of(name)
        assert bench.profile_matches_width(k, 4), k
        assert not bench.profile_matches_width(k, 2), k


def test_width_check_reads_the_template_not_the_arguments():
    assert bench.profile_matches_width("void adgi::trace_shade_kernel<0, false, true>(adgi::VolumeView)", 4)
    assert bench.profile_matches_width("void adgi::trace_hit_kernel<1, true, false>(adgi::VolumeView, int)", 2)
    assert not bench.profile_matches_width("void adgi::blend_wave_kernel(adgi::VolumeView)", 4)
