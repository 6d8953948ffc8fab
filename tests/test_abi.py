"""CPU checks of the C-ABI library: it loads, exports every symbol that
include/art.h declares, and its error strings resolve (no GPU calls)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "art.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(art_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    from paper_1711_06277_amd import _abi as A
    lib = A.lib()
    names = declared_functions()
    assert set(names) == set(A.EXPORTED), names
    for n in names:
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", A.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {line.split()[-1] for line in out.splitlines()}
    assert set(names) <= exported


def test_error_strings():
    from paper_1711_06277_amd import _abi as A
    assert A.strerror(A.ART_OK) == "ok"
    for code in range(-10, 0):
        assert A.strerror(code) != "unknown error"
    assert A.strerror(-99) == "unknown error"


def test_struct_layouts_match_header():
    """ctypes mirrors of the ABI structs have the sizes the C compiler gives."""
    import ctypes as C
    import tempfile
    from paper_1711_06277_amd import _abi as A
    src = ('#include "art.h"\n#include <stdio.h>\nint main(){printf("%zu %zu %zu\\n",'
           'sizeof(art_params),sizeof(art_options),sizeof(art_stats));return 0;}\n')
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "s.c")
        exe = os.path.join(d, "s")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), "-o", exe, c])
        sizes = [int(x) for x in subprocess.check_output([exe]).split()]
    assert sizes == [C.sizeof(A.art_params), C.sizeof(A.art_options), C.sizeof(A.art_stats)]


def test_create_without_gpu_fails_cleanly():
    """With no device, art_create returns an error code instead of crashing."""
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_1711_06277_amd import _abi as A
    p = A.art_params()
    p.level0, p.level_max, p.phi_c, p.tau_term, p.s_H, p.n_bins = 2, 13, 4.0, 23.0, 0.1, 1
    p.rot[0] = p.rot[4] = p.rot[8] = 1.0
    o = A.art_options()
    o.max_sources = 1
    with pytest.raises(A.ArtError):
        A.art_create(8, 8, 8, p, o, 0)
    o.max_sources = 0
    with pytest.raises(A.ArtError) as e:
        A.art_create(8, 8, 8, p, o, 0)
    assert e.value.code == A.ART_ERR_INVALID_ARG
    # termination depths must stay below the cap on a segment's increment
    o.max_sources = 1
    for bad in (5.0e5, 1.0e30, float("inf"), float("nan"), 0.0):
        p.tau_term = bad
        with pytest.raises(A.ArtError) as e:
            A.art_create(8, 8, 8, p, o, 0)
        assert e.value.code == A.ART_ERR_INVALID_ARG, bad


def test_noalloc_rejects_inputs_beyond_its_workspace():
    """art_trace_noalloc checks the sizes against its static workspace before it
    touches a device: a grid whose fixed parts cannot fit is refused with
    ART_ERR_TOO_LARGE (the pointers are never read)."""
    import ctypes as C
    from paper_1711_06277_amd import _abi as A
    p = A.art_params()
    p.level0, p.level_max, p.phi_c, p.tau_term, p.s_H, p.n_bins = 2, 13, 4.0, 23.0, 0.1, 1
    p.rot[0] = p.rot[4] = p.rot[8] = 1.0
    fake = C.c_void_p(256)
    n = 1024  # 76 bytes per cell alone exceed the workspace
    with pytest.raises(A.ArtError) as e:
        A.art_trace_noalloc(n, n, n, p, fake, fake, fake, fake, 1, fake, fake, None, None, 0)
    assert e.value.code == A.ART_ERR_TOO_LARGE
    with pytest.raises(A.ArtError) as e:  # null fields
        A.art_trace_noalloc(8, 8, 8, p, None, fake, fake, fake, 1, fake, fake, None, None, 0)
    assert e.value.code == A.ART_ERR_INVALID_ARG


def test_c_program_links_and_calls_the_library():
    """A C99 program that includes the header, takes the address of every
    declared function, links against libart.so and calls art_strerror: the ABI
    is usable from C without Python (no GPU call is made)."""
    import tempfile
    from paper_1711_06277_amd import _abi as A
    names = declared_functions()
    src = ['#include "art.h"', "#include <stdio.h>", "#include <string.h>", "typedef void (*fn)(void);",
           "int main(void) {", "    fn all[] = {"]
    src += [f"        (fn){n}," for n in names]
    src += ["    };", "    for (unsigned i = 0; i < sizeof all / sizeof all[0]; ++i) if (!all[i]) return 1;",
            '    printf("%s|%s\\n", art_strerror(ART_ERR_QUEUE_OVERFLOW), art_strerror(ART_OK));',
            "    return 0;", "}"]
    libdir = os.path.dirname(A.LIB_PATH)
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "use_art.c")
        exe = os.path.join(d, "use_art")
        open(c, "w").write("\n".join(src) + "\n")
        subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-Wno-cast-function-type",
                               "-I", os.path.join(ROOT, "include"), "-o", exe, c,
                               "-L", libdir, "-l:" + os.path.basename(A.LIB_PATH),
                               "-Wl,-rpath," + libdir, "-Wl,-rpath-link,/opt/rocm/lib"])
        out = subprocess.check_output([exe], text=True).strip()
    assert out == f"{A.strerror(A.ART_ERR_QUEUE_OVERFLOW)}|ok"
