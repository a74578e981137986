"""The committed rocprofv3 summaries under profiles/ describe the kernels as they are built
now: every kernel whose HBM traffic bench.py reports carries the SHA-256 of its sources in
its PMC summary, and that hash matches the sources in the tree (otherwise bench.py's
`traffic` fields would go null without notice).  Every summary states the command that
produced it."""
import os

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _summary_of(kernel):
    return "fmg2d_n2048_pmc.md" if ("2d" in kernel or "<2>" in kernel) else "fmg3d_n256_pmc.md"


def test_pmc_summaries_match_the_kernel_sources():
    stale = [k for k, src in bench.PMC_KERNELS.items() if bench._pmc_traffic(_summary_of(k), k, src) is None]
    assert not stale, f"PMC summaries taken before the last change to these kernels' sources: {stale}"


def test_every_profile_summary_states_its_command():
    folder = os.path.join(ROOT, "profiles")
    names = sorted(f for f in os.listdir(folder) if f.endswith(".md"))
    assert names
    for name in names:
        text = open(os.path.join(folder, name)).read()
        assert "rocprofv3 " in text, name
        assert "Command" in text, name
