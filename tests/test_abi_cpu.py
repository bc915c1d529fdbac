"""The C ABI library loads, exports every entry point of include/ngdbf.h,
and rejects invalid arguments on the host (no GPU needed for these paths)."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_1402_2773_amd as ng

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def L():
    if not os.path.exists(ng.LIB_PATH):
        from paper_1402_2773_amd import build

        build.build()
    return ng.lib()


def _declared():
    with open(os.path.join(ROOT, "include", "ngdbf.h")) as f:
        src = f.read()
    return sorted(set(re.findall(r"^(?:ngdbf_status|const char \*)\s*(ngdbf_\w+)\s*\(", src, re.M)))


def test_header_declares_the_binding_functions():
    assert sorted(ng.ABI_FUNCTIONS) == _declared()


def test_library_exports_every_declared_symbol(L):
    for name in _declared():
        assert hasattr(L, name), name


def test_build_compiles_every_source_and_decoder_family():
    """Every HIP/C++ source under csrc is a build unit, and the extended
    decoder source is compiled once per family (the library holds all four
    families' dispatchers)."""
    from paper_1402_2773_amd import build

    csrc = os.path.join(ROOT, "paper_1402_2773_amd", "csrc")
    sources = {f for f in os.listdir(csrc) if f.endswith((".hip", ".cpp"))}
    assert sources == {u[0] for u in build.UNITS}
    fams = sorted(x for src, flags, _ in build.UNITS if src == "decode_ext.hip" for x in flags)
    assert fams == [f"-DNGDBF_EXT_FAMILY={k}" for k in range(4)]
    assert len({u[2] for u in build.UNITS}) == len(build.UNITS)  # one object name each


def test_create_code_rejects_bad_tables(L):
    with pytest.raises(ng.NgdbfError, match="row_ptr"):
        ng.ngdbf_create_code(4, 2, [1, 2, 4], [0, 1, 2, 3])
    with pytest.raises(ng.NgdbfError, match="out of range"):
        ng.ngdbf_create_code(4, 2, [0, 2, 4], [0, 1, 2, 9])
    with pytest.raises(ng.NgdbfError, match="repeats"):
        ng.ngdbf_create_code(4, 2, [0, 2, 4], [0, 0, 2, 3])
    with pytest.raises(ng.NgdbfError, match="empty"):
        ng.ngdbf_create_code(4, 2, [0, 2, 2], [0, 1])
    with pytest.raises(ng.NgdbfError, match="column 3 is empty"):
        ng.ngdbf_create_code(4, 2, [0, 2, 3], [0, 1, 2])
    with pytest.raises(ng.NgdbfError, match="m < n"):
        ng.ngdbf_create_code(2, 2, [0, 1, 2], [0, 1])


def test_decode_rejects_null_code(L):
    p = ng.Params().c(ng.NGDBF_Y_F32)
    with pytest.raises(ng.NgdbfError, match="code is NULL"):
        ng.ngdbf_decode(None, None, 0, None, 0.5, p, 1, 0, None, None, None, 0)
    assert ng.ngdbf_last_error() == "code is NULL"


def test_noise_probe_rejects_bad_ranges(L):
    buf = np.zeros(4, dtype=np.float32)
    with pytest.raises(ng.NgdbfError, match="unknown probe kind"):
        ng.ngdbf_noise_probe(7, 0, 1, 0, 0, 0, buf, None, 0)
    with pytest.raises(ng.NgdbfError, match="radius probe range"):
        ng.ngdbf_noise_probe(0, 0, 1, 0, 0, 0, buf, None, 0)
    with pytest.raises(ng.NgdbfError, match="angle probe range"):
        ng.ngdbf_noise_probe(1, (1 << 24) - 1, 2, 0, 0, 0, buf, buf, 0)


def test_issue_probe_rejects_bad_arguments(L):
    # every check happens before anything touches a device
    buf = np.zeros(256, dtype=np.uint32)
    for kind, blocks, iters, out in [(-1, 1, 1, buf), (28, 1, 1, buf), (0, 0, 1, buf), (0, 1, 0, buf),
                                     (0, 1, 1, None)]:
        st = L.ngdbf_issue_probe(kind, blocks, iters, out.ctypes.data if out is not None else None, None)
        assert st == ng.NGDBF_EINVAL


def test_params_struct_layout_matches_header():
    assert ctypes.sizeof(ng.ngdbf_params) == 44
    names = [f[0] for f in ng.ngdbf_params._fields_]
    assert names == ["w", "theta", "lam", "eta", "ymax", "t_max", "smooth_window", "y_format",
                     "variant", "quant_bits", "noise_reuse"]


def test_batch_and_shape_reject_bad_arguments(L):
    with pytest.raises(ng.NgdbfError, match="bad job array"):
        L_status = ng.lib().ngdbf_decode_batch(None, -1, None)
        ng._check(L_status)
    with pytest.raises(ng.NgdbfError, match="code is NULL"):
        ng.ngdbf_code_set_shape(None, 1, 4, 8)
    with pytest.raises(ng.NgdbfError, match="code is NULL"):
        ng.ngdbf_code_set_stats(None, None)
    p = ng.Params().c(ng.NGDBF_Y_F32)
    bad = ng.ngdbf_job(None, None, 0, None, 0.5, p, 1, 0, None, None, None)
    with pytest.raises(ng.NgdbfError, match="job 0: code is NULL"):
        ng.ngdbf_decode_batch([bad], 0)


def test_server_rejects_bad_arguments(L):
    p = ng.Params().c(ng.NGDBF_Y_F32)
    with pytest.raises(ng.NgdbfError, match="codes, params and pool sizes"):
        ng.ngdbf_server_create([], [], [], 1, 16, 1)
    with pytest.raises(ng.NgdbfError, match="n_streams"):
        ng.ngdbf_server_create([None], [p], [16], 0, 16, 1)
    with pytest.raises(ng.NgdbfError, match="max_requests_per_launch"):
        ng.ngdbf_server_create([None], [p], [16], 1, 0, 1)
    with pytest.raises(ng.NgdbfError, match="launches_per_stream"):
        ng.ngdbf_server_create([None], [p], [16], 4, 16, 17)
    for call in (lambda: ng.ngdbf_server_pump(None), lambda: ng.ngdbf_server_poll(None, 4),
                 lambda: ng.ngdbf_server_release(None, [1]), lambda: ng.ngdbf_server_commit(None, [1], 0),
                 lambda: ng.ngdbf_server_pools(None, 0)):
        with pytest.raises(ng.NgdbfError):
            call()


def test_segments_require_a_table(L):
    p = ng.Params().c(ng.NGDBF_Y_F32)
    with pytest.raises(ng.NgdbfError, match="segments are required"):
        ng.ngdbf_decode_segments(None, None, None, 0.5, 8, p, None, 0, 4, None, None, None, 0)


def test_params_validation_of_the_extended_decoders(L):
    """Parameters are checked on the host before anything else."""
    base = ng.Params()
    for bad, msg in ((dict(variant=3), "unknown variant"), (dict(quant_bits=9), "quant_bits"),
                     (dict(quant_bits=3, ymax=0.0), "finite ymax"),
                     (dict(quant_bits=3, variant=2), "mode switching"),
                     (dict(noise_reuse=2), "noise_reuse")):
        p = ng.Params(**{**base.__dict__, **bad}).c(ng.NGDBF_Y_F32)
        with pytest.raises(ng.NgdbfError, match=msg):
            ng.ngdbf_decode(None, None, 0, None, 0.5, p, 1, 0, None, None, None, 0)


def test_objective_rejects_bad_arguments(L):
    with pytest.raises(ng.NgdbfError, match="code is NULL"):
        ng.ngdbf_objective(None, None, 0, 1, 2.5, None, None, 0)


@pytest.mark.parametrize("sigma", [-0.5, float("nan"), float("inf")])
def test_decode_rejects_bad_sigma(L, sigma):
    p = ng.Params().c(ng.NGDBF_Y_F32)
    with pytest.raises(ng.NgdbfError, match="sigma_scalar"):
        ng.ngdbf_decode(None, None, 4, None, sigma, p, 1, 0, None, None, None, 0)


def test_decode_rejects_negative_frames_and_bad_params(L):
    p = ng.Params().c(ng.NGDBF_Y_F32)
    with pytest.raises(ng.NgdbfError, match="n_frames < 0"):
        ng.ngdbf_decode(None, None, -1, None, 0.5, p, 1, 0, None, None, None, 0)
    for bad, msg in ((dict(t_max=-1), "t_max"), (dict(lam=0.0), "lambda"), (dict(lam=1.5), "lambda"),
                     (dict(w=0.0), "w must"), (dict(eta=-1.0), "eta"),
                     (dict(theta=float("nan")), "theta"), (dict(smooth_window=-2), "smooth_window")):
        q = ng.Params(**{**ng.Params().__dict__, **bad}).c(ng.NGDBF_Y_F32)
        with pytest.raises(ng.NgdbfError, match=msg):
            ng.ngdbf_decode(None, None, 4, None, 0.5, q, 1, 0, None, None, None, 0)
    q = ng.Params().c(7)
    with pytest.raises(ng.NgdbfError, match="unknown y_format"):
        ng.ngdbf_decode(None, None, 4, None, 0.5, q, 1, 0, None, None, None, 0)


def test_create_code_rejects_more_shapes(L):
    with pytest.raises(ng.NgdbfError, match="row_ptr\\[0\\]"):
        ng.ngdbf_create_code(4, 2, [1, 2, 4], [0, 1, 2, 3])
    with pytest.raises(ng.NgdbfError, match="need 1 <= m < n"):
        ng.ngdbf_create_code(70000, 2, [0, 1, 2], [0, 1])


def _struct_fields(path, name):
    """(type, field) pairs of `typedef struct { ... } name;` in a C header."""
    with open(path) as f:
        src = f.read()
    body = re.search(r"typedef struct \{(.*?)\}\s*" + name + r"\s*;", src, re.S).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    return [tuple(m) for m in re.findall(r"(float|int32_t)\s+(\w+)\s*;", body)]


def test_oracle_params_agree_with_the_abi_params_field_by_field():
    """The oracle's parameter block (oracle/ngdbf_oracle.h) and the ABI's
    (include/ngdbf.h) hold the same fields with the same C types in the same
    order; the ABI's one extra field, y_format, is a separate argument of the
    oracle's decode.  The two Python mirrors carry the same values into them."""
    import oracle

    abi = _struct_fields(os.path.join(ROOT, "include", "ngdbf.h"), "ngdbf_params")
    ref = _struct_fields(os.path.join(ROOT, "oracle", "ngdbf_oracle.h"), "ngdbf_ref_params")
    assert [f for f in abi if f[1] != "y_format"] == ref
    assert ("int32_t", "y_format") in abi
    # the ctypes mirrors follow their headers (lambda is spelled lam in Python)
    py = lambda n: "lam" if n == "lambda" else n  # noqa: E731
    assert [f[0] for f in ng.ngdbf_params._fields_] == [py(n) for _, n in abi]
    assert [f[0] for f in oracle._Params._fields_] == [py(n) for _, n in ref]
    for (t, n), (fname, ctype) in zip(abi, ng.ngdbf_params._fields_):
        assert ctype == (ctypes.c_float if t == "float" else ctypes.c_int32), n
    # the same parameter values reach both structures
    gp = ng.Params(w=0.5, theta=0.25, lam=0.875, eta=1.5, ymax=2.0, t_max=77, smooth_window=9,
                   variant=1, quant_bits=3, noise_reuse=1)
    assert dataclasses_fields(gp) == dataclasses_fields(oracle.Params())
    rp = oracle.Params(**gp.__dict__)
    gc, rc = gp.c(ng.NGDBF_Y_I8), rp.c()
    for fname, _ in oracle._Params._fields_:
        assert getattr(gc, fname) == getattr(rc, fname), fname
    assert gc.y_format == ng.NGDBF_Y_I8


def dataclasses_fields(obj):
    import dataclasses

    return [f.name for f in dataclasses.fields(obj)]


def test_create_code_checks_nnz(L):
    with pytest.raises(ng.NgdbfError, match="differs from nnz"):
        ng.ngdbf_create_code(4, 2, [0, 2, 4], [0, 1, 2, 3], nnz=5)
    with pytest.raises(ng.NgdbfError, match="exceeds nnz"):
        ng.ngdbf_create_code(4, 2, [0, 2, 4], [0, 1, 2, 3], nnz=3)
    with pytest.raises(ng.NgdbfError, match="every one of the 2 rows"):
        ng.ngdbf_create_code(4, 2, [0, 2, 4], [0, 1, 2, 3], nnz=1)


def test_batch_may_not_wrap_the_queue_ring(L):
    """Every job of a batch takes its own frame queue before any is launched,
    so a batch larger than the ring of 1024 queues is refused up front."""
    p = ng.Params().c(ng.NGDBF_Y_F32)
    jobs = [ng.ngdbf_job(None, None, 0, None, 0.5, p, 1, 0, None, None, None)] * 1025
    with pytest.raises(ng.NgdbfError, match="1025 jobs exceed the 1024 frame queues") as e:
        ng.ngdbf_decode_batch(jobs, 0)
    assert e.value.status == ng.NGDBF_EINVAL
