"""Host-side checks of the C ABI (no GPU needed): the library builds for gfx950,
loads, exports every entry point the header declares, the ctypes mirror of
each structure matches the header's layout, and argument validation that
happens before any device call rejects bad input."""
import ctypes
import os
import re
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "compacttag.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2311_04406_amd import binding, build
    if not os.path.exists(binding.LIB_PATH):
        build.build()
    return binding.load()


def declared_functions():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:ct_status|const char \*|double)\s*(ct_\w+)\s*\(", src, re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for f in ("ct_create", "ct_destroy", "ct_gen_triple_tags", "ct_tag_linear", "ct_mac_check",
              "ct_mac_check_device", "ct_key_shares", "ct_last_error", "ct_plan_create", "ct_plan_launch",
              "ct_plan_destroy", "ct_server_create", "ct_server_submit", "ct_server_poll", "ct_server_drain",
              "ct_server_layer", "ct_server_stats", "ct_server_destroy", "ct_server_now_us"):
        assert f in names


def test_every_declared_symbol_is_exported(lib):
    from paper_2311_04406_amd import binding
    out = subprocess.run(["nm", "-D", "--defined-only", binding.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\sT\s(ct_\w+)$", out, re.M))
    for f in declared_functions():
        assert f in exported, f
        assert hasattr(lib, f)


def test_library_is_built_for_gfx950():
    from paper_2311_04406_amd import binding
    data = open(binding.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_struct_layouts_match_header():
    from paper_2311_04406_amd import binding as b
    prog = r"""
#include <stdio.h>
#include <stddef.h>
#include "compacttag.h"
int main(void) {
  printf("%zu %zu %zu %zu\n", sizeof(ct_params), sizeof(ct_layer_desc), sizeof(ct_layer_bufs), sizeof(ct_check_result));
  printf("%zu %zu %zu %zu\n", offsetof(ct_params, hip_stream), offsetof(ct_params, max_layers),
         offsetof(ct_layer_desc, seed), offsetof(ct_layer_desc, layer_id));
  printf("%zu %zu %zu %zu %zu\n", offsetof(ct_layer_bufs, E), offsetof(ct_layer_bufs, cvec), offsetof(ct_check_result, accept),
         offsetof(ct_layer_bufs, Rf), offsetof(ct_layer_bufs, tZf));
  printf("%zu %zu %zu %zu\n", sizeof(ct_server_params), sizeof(ct_request), sizeof(ct_completion), sizeof(ct_server_counts));
  printf("%zu %zu %zu %zu %zu %zu %zu\n", offsetof(ct_server_params, mode), offsetof(ct_request, layer),
         offsetof(ct_request, arrival_us), offsetof(ct_completion, done_us), offsetof(ct_completion, result),
         offsetof(ct_server_counts, arena_bytes), offsetof(ct_server_counts, arena_used));
  printf("%zu %zu %zu %d\n", offsetof(ct_layer_desc, compress), offsetof(ct_layer_desc, conv_pad),
         offsetof(ct_params, parties), CT_MAX_PARTIES);
  {
    const long long sh[3][3] = {{64, 576, 3136}, {7, 9, 7}, {4096, 25088, 1}};
    for (int i = 0; i < 3; i++)
      for (int n = 2; n <= CT_MAX_PARTIES; n++)
        printf("%lld %lld ", (long long)CT_WORK_LEN_NP(sh[i][0], sh[i][1], sh[i][2], n),
               (long long)CT_CVEC_LEN_NP(sh[i][0], sh[i][1], n));
    printf("\n");
  }
  {
    const long long sh[4][3] = {{4096, 25088, 1}, {64, 576, 3136}, {7, 9, 7}, {3, 5, 2}};
    for (int i = 0; i < 4; i++)
      for (int c = 0; c < 3; c++)
        printf("%lld ", (long long)CT_CVEC_LEN_FOR(sh[i][0], sh[i][1], sh[i][2], c));
    printf("\n");
  }
  return 0;
}
"""
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "l.c")
        open(c, "w").write(prog)
        exe = os.path.join(d, "l")
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        vals = [int(x) for x in subprocess.check_output([exe]).split()]
    got = [ctypes.sizeof(b.CtParams), ctypes.sizeof(b.CtLayerDesc), ctypes.sizeof(b.CtLayerBufs),
           ctypes.sizeof(b.CtCheckResult),
           b.CtParams.hip_stream.offset, b.CtParams.max_layers.offset, b.CtLayerDesc.seed.offset,
           b.CtLayerDesc.layer_id.offset, b.CtLayerBufs.E.offset, b.CtLayerBufs.cvec.offset,
           b.CtCheckResult.accept.offset, b.CtLayerBufs.Rf.offset, b.CtLayerBufs.tZf.offset,
           ctypes.sizeof(b.CtServerParams), ctypes.sizeof(b.CtRequest), ctypes.sizeof(b.CtCompletion),
           ctypes.sizeof(b.CtServerCounts),
           b.CtServerParams.mode.offset, b.CtRequest.layer.offset, b.CtRequest.arrival_us.offset,
           b.CtCompletion.done_us.offset, b.CtCompletion.result.offset, b.CtServerCounts.arena_bytes.offset,
           b.CtServerCounts.arena_used.offset, b.CtLayerDesc.compress.offset, b.CtLayerDesc.conv_pad.offset,
           b.CtParams.parties.offset, b.MAX_PARTIES]
    for M, K, N in ((64, 576, 3136), (7, 9, 7), (4096, 25088, 1)):
        for n in range(2, b.MAX_PARTIES + 1):
            got += [b.work_len(M, K, N, n), (1 + n) * K + (2 + 4 * n) * M]
    got += [b.cvec_len(M, K, N, c) for M, K, N in ((4096, 25088, 1), (64, 576, 3136), (7, 9, 7), (3, 5, 2))
            for c in range(3)]
    assert got == vals


def test_validation_before_device_calls(lib):
    from paper_2311_04406_amd import binding as b
    h = ctypes.c_void_p()
    # parameter sets other than k = s = 64 and k = s = 32 are rejected before the device is touched
    for kb, sb in ((32, 64), (64, 32), (16, 16), (48, 48)):
        p = b.CtParams(0, 1, kb, sb, None, 4)
        assert lib.ct_create(ctypes.byref(h), ctypes.byref(p)) == b.CT_EINVAL
    # party counts outside 2 .. CT_MAX_PARTIES
    for parties in (1, -1, b.MAX_PARTIES + 1):
        p = b.CtParams(0, 1, 64, 64, None, 4, parties)
        assert lib.ct_create(ctypes.byref(h), ctypes.byref(p)) == b.CT_EINVAL
    assert lib.ct_create(None, ctypes.byref(p)) == b.CT_EINVAL
    assert lib.ct_destroy(None) == b.CT_EINVAL
    assert lib.ct_key_shares(None, None) == b.CT_EINVAL
    assert lib.ct_tag_linear(None, 1, None, None, 1) == b.CT_EINVAL
    assert lib.ct_mac_check(None, 1, None, None, 1, None) == b.CT_EINVAL
    assert lib.ct_gen_triple_tags(None, None, None, 1, 1) == b.CT_EINVAL
    assert lib.ct_last_error(None) == b"null context"
    assert lib.ct_plan_create(None, 1, None, None, 1, None, None) == b.CT_EINVAL
    assert lib.ct_plan_launch(None) == b.CT_EINVAL
    assert lib.ct_plan_destroy(None) == b.CT_EINVAL
    assert lib.ct_server_create(None, None, None) == b.CT_EINVAL
    assert lib.ct_server_submit(None, None, 0) == b.CT_EINVAL
    assert lib.ct_server_poll(None, None, 0, None) == b.CT_EINVAL
    assert lib.ct_server_drain(None, 1.0) == b.CT_EINVAL
    assert lib.ct_server_destroy(None) == b.CT_EINVAL
    assert lib.ct_server_last_error(None) == b"null server"
    assert lib.ct_set_launch(None, b.LAUNCH_STAGED) == b.CT_EINVAL
    assert lib.ct_set_launch_wait(None, b.LAUNCH_WAIT_DEFAULT) == b.CT_EINVAL
    assert lib.ct_set_overlap(None, 1) == b.CT_EINVAL


def test_product_path_has_no_oracle_dependency():
    """The package never imports or links the oracle (no CPU fallback)."""
    pkg = os.path.join(ROOT, "paper_2311_04406_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in src and "from oracle" not in src, f
                assert "ct_oracle" not in src, f
