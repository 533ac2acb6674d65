"""The stage kernels load the next chunk into LDS, the FP64 x-flux kernels
the next segment into registers, and both then wait with s_waitcnt vmcnt(N),
N = the stores of the current chunk or segment, so that those stores stay in
flight; the y/z window kernels wait for a ring row with vmcnt(32) (34 with a
shift, 29 on a flat metric) and for the rhs row they read with vmcnt(7).
That wait is only safe if every path from the last load into LDS to the wait
issues at least N vector-memory instructions (vmcnt counts them in order).
Inside the loops of the x and window kernels no wait may be a full
vmcnt(0), which would stall each step on every load in flight.  Compiles the kernels for gfx950 and checks it on the
control-flow graph of their assembly (no device needed)."""
import os
import re
import shutil
import subprocess

import pytest

from asmcheck.vmcount import kernels, path_counts

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.fixture(scope="module")
def asm(tmp_path_factory):
    if not os.path.exists(HIPCC) and not shutil.which("hipcc"):
        pytest.skip("hipcc not available")
    out = tmp_path_factory.mktemp("asm") / "stage.s"
    cmd = [HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2510_18968_amd", "csrc"), "--cuda-device-only", "-S",
           os.path.join(ROOT, "tests", "asmcheck", "stage_kernels.hip"), "-o", str(out)]
    subprocess.run(cmd, check=True, capture_output=True)
    return kernels(out.read_text())


@pytest.mark.parametrize("kind,count,load", [("k_stage", 20, "global_load_lds_dwordx4"),
                                             ("k_flux_p", 9, "global_load_dwordx2")])
def test_kernel_waits_cover_their_loads(asm, kind, count, load):
    ks = {k: v for k, v in asm.items() if kind in k}
    assert len(ks) == count
    for name, L in ks.items():
        lds = [i for i, l in enumerate(L) if load in l]
        waits = [(i, int(m.group(1))) for i, l in enumerate(L)
                 for m in [re.search(r's_waitcnt vmcnt\((\d+)\)', l)] if m and int(m.group(1)) > 0]
        assert lds and waits, name
        # the loop's loads are the last block of loads; every nonzero vmcnt
        # wait reachable from them must be covered
        last = lds[-1]
        checked = 0
        for wi, n in waits:
            lo, hi = path_counts(L, last + 1, wi)
            if lo is None:
                continue
            print(f"{name[:40]}: vmcnt({n}) after the loop loads: {lo}..{hi} vector-memory ops on the way")
            assert lo >= n, (name, n, lo)
            checked += 1
        assert checked >= 1, name


def test_window_kernel_waits_cover_their_loads(asm):
    ks = {k: v for k, v in asm.items() if "k_flux_w" in k}
    assert len(ks) == 15
    for name, L in ks.items():
        m = re.search(r"k_flux_wILi(\d)ELi(\d)ELb(\d)E([df])Lb(\d)ELb(\d)ELb(\d)E", name)
        curved, shift, diag = m.group(3) == "1", m.group(5) == "1", m.group(6) == "1"
        fuse = m.group(7) == "1"
        # the step's stores (rhs row, or the stage update's 32), the staging
        # row (sigma, alpha, gamma_ij -- its diagonal on a diagonal metric --,
        # beta^i, in pairs), rhs reads
        nstage = (2 + (3 if diag else 6) + (3 if shift else 0) + 1) // 2 if curved else 1
        # (fused: the update's 17 loads too; vmcnt holds at most 63)
        n_ring = min(63, 32 + nstage + 14 + 17) if fuse else 14 + nstage + 14
        dma = [i for i, l in enumerate(L) if "global_load_lds_dwordx4" in l]
        heads = [i for i, l in enumerate(L) if "Loop Header" in l and i < dma[-1]]
        assert dma and heads, name
        # ring rows: every path from the loop's last ring load to the ring wait
        ring_waits = [i for i, l in enumerate(L) if re.search(rf"s_waitcnt vmcnt\({n_ring}\)", l)]
        assert ring_waits, (name, n_ring)
        for w in ring_waits:
            lo, hi = path_counts(L, dma[-1] + 1, w)
            print(f"{name[:44]}: vmcnt({n_ring}) after the ring load: {lo}..{hi}")
            assert lo is not None and lo >= n_ring, (name, lo)
        if fuse:
            # the rhs row and the update's U^n and R1 rows at the top of the
            # step, then the wait before the update (ring row c + 3 behind them)
            loads = [i for i, l in enumerate(L) if "global_load_dwordx2" in l and i > heads[-1]][:31]
            waits = [i for i, l in enumerate(L) if "s_waitcnt vmcnt(7)" in l and i > loads[-1]]
            assert len(loads) == 31 and waits, (name, len(loads))
            for w in waits:
                lo, hi = path_counts(L, loads[-1] + 1, w)
                print(f"{name[:44]}: vmcnt(7) after the update's loads: {lo}..{hi}")
                assert lo is not None and lo >= 7, (name, lo)
            continue
        # rhs row: the 14 loads after the loop head, then the wait before the stores
        rhs = [i for i, l in enumerate(L) if "global_load_dwordx2" in l and i > heads[-1]][:14]
        rhs_waits = [i for i, l in enumerate(L) if "s_waitcnt vmcnt(7)" in l and i > rhs[-1]]
        assert len(rhs) == 14 and rhs_waits, name
        for w in rhs_waits:
            lo, hi = path_counts(L, rhs[-1] + 1, w)
            print(f"{name[:44]}: vmcnt(7) after the rhs loads: {lo}..{hi}")
            assert lo is not None and lo >= 7, (name, lo)


def loop_full_waits(L):
    """Lines in loop blocks (the compiler's "in Loop" label comments) that wait
    for every vector memory op.  Not counted: a wait right before an LDS
    atomic of the fused window's stage tally, which sits in the same LDS
    object as the ring and runs only on a failed cell or with the iteration
    histogram on."""
    hits, inloop = [], False
    for i, l in enumerate(L):
        if re.match(r"^(\.LBB\S+:|; %bb\.\d+:)", l):
            inloop = "Loop" in l
        if inloop and re.search(r"s_waitcnt\s.*vmcnt\(0\)", l):
            if i + 1 < len(L) and "ds_add_u32" in L[i + 1]:
                continue
            hits.append(i)
    return hits


def test_no_full_wait_inside_sweep_loops(asm):
    ks = {k: v for k, v in asm.items() if "k_flux_w" in k or "k_flux_p" in k}
    assert len(ks) == 24
    checked = 0
    for name, L in ks.items():
        if any("scratch_" in l for l in L):
            continue            # register spills are reloaded with full waits (the WENO5 FP64 shift variant)
        assert not loop_full_waits(L), name
        checked += 1
    assert checked >= 18
