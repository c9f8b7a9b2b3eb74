"""Every pipeline kernel after the grid build returns when an input error is flagged (CPU, on
the kernel sources).

The refinement kernels leave their tables unwritten when an error is already set, so any later
kernel that walked them would read memory no kernel of the call wrote (a fresh context's
uninitialised memory).  The status word is only ever set during a call and every kernel runs
after the previous one on the stream, so one check at a kernel's start rules that out.  Only
the grid build itself (clear, prep, scatter and the bucket scan, which run unconditionally and
write every entry they and the scan read) is exempt.
"""
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "paper_1212_1095_amd", "csrc", "vor_kernels.hip")
EXEMPT = {"k_clear", "k_prep", "k_scatter"}
GATE = re.compile(r"if \((gate && )?\*status( & \([A-Z_| ]+\))?\) return;|stop = \*status;")


def kernels():
    src = open(SRC).read()
    out = {}
    for m in re.finditer(r"__global__[^{;]*?\b(k_\w+)\s*\(", src):
        name = m.group(1)
        body_start = src.index("{", m.end())
        depth, i = 0, body_start
        while True:
            if src[i] == "{":
                depth += 1
            elif src[i] == "}":
                depth -= 1
                if depth == 0:
                    break
            i += 1
        out[name] = src[body_start + 1:i]
    return out


def test_every_kernel_after_the_grid_build_checks_the_status_first():
    ks = kernels()
    assert EXEMPT <= set(ks), "the exempt kernels exist"
    assert len(ks) >= 14
    for name, body in ks.items():
        if name in EXEMPT:
            continue
        m = GATE.search(body)
        assert m, f"{name} never checks the status word"
        head = body[:m.start()]
        # before the check: declarations of shared memory and index arithmetic only, no loads
        # through pointer arguments (no '[' indexing and no loop)
        code = "\n".join(l for l in head.splitlines() if "__shared__" not in l)
        assert "[" not in code and "for (" not in code and "while" not in code, \
            f"{name} reads memory before its status check:\n{code}"


def test_scan_gate_is_set_except_for_the_bucket_scan():
    launch = open(SRC).read().split("void launch_stage", 1)[1]
    calls = re.findall(r"launch_scan\(([^;]*)\);", launch)
    assert len(calls) == 4
    ungated = [c for c in calls if re.search(r",\s*0,\s*st\s*$", c)]
    assert len(ungated) == 1 and "a.bstart" in ungated[0], ungated


def test_subwedge_workgroups_have_a_wave_per_corner_ray():
    """The subwedge passes shoot the projector's three corner rays on waves 0, 1 and 2 of a
    workgroup in their first round; a workgroup with fewer waves would leave a corner unwritten
    and follow a garbage successor link in the later rounds."""
    src = open(SRC).read()
    assert "if (wave < 3)" in src
    for name in ("WIDE_WAVES", "WIDE_LWAVES"):
        m = re.search(r"constexpr int %s = (\d+);" % name, src) or re.search(
            r"constexpr int %s = (\d+);" % name,
            open(os.path.join(ROOT, "paper_1212_1095_amd", "csrc", "vor_internal.h")).read())
        assert m, name
        assert int(m.group(1)) >= 3, name
