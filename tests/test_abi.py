"""The C-ABI library loads on a machine without a GPU and exports every
function that include/tlvlbm.h declares (no compute call is made)."""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "tlvlbm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(tlvlbm_[a-z_]+)\s*\(", txt)))


def test_library_exports_declared_symbols():
    from paper_2606_20646_amd import LIB_PATH
    lib = ctypes.CDLL(LIB_PATH)
    names = _declared()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def test_product_path_does_not_reference_the_oracle():
    pkg = os.path.join(ROOT, "paper_2606_20646_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in src and "orc_" not in src, f


def test_default_options_are_the_papers_settings():
    from paper_2606_20646_amd import tlvlbm as T
    o = T.Options()
    T.lib.tlvlbm_default_options(ctypes.byref(o))
    assert (o.omega, o.theta_F, o.proj_every, o.track_u) == (1.8, 1.0, 20, -1)


def test_bulk_kernel_bodies_in_sync():
    """The single-instance bulk kernel carries the update inline (faster
    code than the shared device function); both bodies must stay identical
    apart from how the node position is obtained and the tape block."""
    src = open(os.path.join(ROOT, "paper_2606_20646_amd", "csrc", "bulk.hip")).read()

    def body(start):
        i = src.index("{", src.index(start)) + 1
        j = src.index("\n}\n", i)
        return [l.rstrip() for l in src[i:j].splitlines() if l.strip()]

    kern = body("void k_bulk(const T *__restrict__ fin")
    node = body("void bulk_node(const T *__restrict__ fin")
    kern = [l for l in kern if l.strip() not in ("const int x = blockIdx.x * blockDim.x + threadIdx.x;",
                                                 "if (x >= g.nx) return;", "const int row = blockIdx.y;")]
    out, skip = [], 0
    for l in node:
        if l.strip() == "if constexpr (TAPE) {":
            skip = 1
            continue
        if skip:
            skip += l.count("{") - l.count("}")
            if l.strip() == "}" and skip == 0:
                continue
            if skip > 0:
                continue
        out.append(l)
    assert kern == out
