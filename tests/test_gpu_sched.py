"""GPU: the persistent scheduler past one wave's scan, and its time limit.

- A batch of more systems than one 64-lane scan covers (wave 0 looks at the
  ticket words in rounds of 64): every system against the oracle, at both
  workgroup sizes.
- The time limit, forced from the host with a limit far below the solve's
  own time: the launch returns early, systems left unfinished report
  ERR_TIMEOUT, finished ones keep their status and solution, and the next
  solve on the same objects starts from a clean state.
"""
import sys
import time

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import csl_oracle as O

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def csl():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2408_00488_amd as C
    C.load_library()
    return C


def _crand(shape, seed):
    g = np.random.default_rng(seed)
    return g.standard_normal(shape) + 1j * g.standard_normal(shape)


def _coef(shape, seed, lo=0.5, hi=2.0):
    return np.random.default_rng(seed).uniform(lo, hi, shape)


def cuda(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def rel(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _vs_oracle(po, lam, f, zg, info, zo, io):
    """Relative difference of the GPU iterate from the oracle's at the GPU's
    iteration count, after checking that the GPU solution is a valid one.

    Shifts close to an eigenvalue of K (small beta, alpha inside the
    spectrum) make MINRES sensitive to rounding: two FP64 runs then differ
    at the 1e-10 level in the iterates, which moves a true residual that sits
    at the tolerance to either side of it, and the stopping step by one or
    two.  What is unique is checked instead: the oracle's own true residual
    of the GPU solution meets the tolerance, and the iterate equals the
    oracle's after the same number of steps.
    """
    r = f - O.apply_A(po.K, lam.real, lam.imag, np.conj(zg))
    assert np.linalg.norm(r) / np.linalg.norm(f) <= 1.01e-8, info
    if info["iters"] == io["iters"]:
        return rel(zg, zo)
    assert abs(info["iters"] - io["iters"]) <= 2, (info, io)
    zf, _ = po.solve(f, fixed_iters=info["iters"])
    return rel(zg, zf)


def _many_systems(count):
    """2-D grids 7..31 and 3-D grids 7, shifts spread over both half planes."""
    shapes = [(7, 7), (15, 15), (31, 31), (15, 31), (7, 7, 7), (7, 15, 7)]
    out = []
    for j in range(count):
        shape = shapes[j % len(shapes)]
        lam = complex(-60.0 + 3.0 * j, 1.0 + 0.5 * (j % 11))
        out.append((shape, _coef(shape, 100 + j), lam, _crand(shape, 200 + j)))
    return out


@pytest.mark.parametrize("block_threads", [256, 512])
def test_batch_more_than_64_systems(csl, block_threads):
    systems = _many_systems(80)
    _say("batch of", len(systems), "block_threads", block_threads)
    probs = [csl.Problem(cuda(a), lam.real, lam.imag, dst="fft") for _, a, lam, _ in systems]
    fs = [cuda(f) for *_, f in systems]
    b = csl.Batch(probs, timeout_ms=30000, block_threads=block_threads)
    assert b.schedule["block_threads"] == block_threads
    zs, infos = b.solve(fs)
    worst = 0.0
    for (shape, a, lam, f), p, z, info in zip(systems, probs, zs, infos):
        assert info["status"] == 0, (shape, lam, info)
        po = O.Problem(a, lam.real, lam.imag)
        zo, io = po.solve(f)
        worst = max(worst, _vs_oracle(po, lam, f, z.cpu().numpy(), info, zo, io))
    _say("worst relative difference", worst)
    assert worst <= 1e-9
    # a replay of the graph gives the same systems the same results, bitwise
    zs2, infos2 = b.solve(fs)
    assert infos2 == infos
    assert all(torch.equal(z, z2) for z, z2 in zip(zs, zs2))
    b.close()
    for p in probs:
        p.close()


# 1024: the plane phase (FP32 preconditioner)
@pytest.mark.parametrize("block_threads", [256, 512, 1024])
def test_time_limit_single(csl, block_threads):
    n = 127
    a = _coef((n, n, n), 7, 1.0, 3.0)
    f = cuda(_crand((n, n, n), 8))
    p = csl.Problem(cuda(a), 10.0, 100.0, dst="fft", pinv_fp32=(block_threads == 1024))
    p.set_schedule(0, 0, block_threads)
    _say("time limit, 3-D", n, "block_threads", block_threads)
    z_full, info_full = csl.minres_solve(p, f, timeout_ms=30000)
    t0 = time.perf_counter()
    z_full, info_full = csl.minres_solve(p, f, timeout_ms=30000)
    t_full = time.perf_counter() - t0
    assert info_full["status"] == 0
    t0 = time.perf_counter()
    z_cut, info_cut = csl.minres_solve(p, f, timeout_ms=1, raise_on_error=False)
    t_cut = time.perf_counter() - t0
    _say("full", info_full["iters"], "iterations in", t_full, "s; limited:", info_cut, t_cut, "s")
    assert info_cut["status_name"] == "ERR_TIMEOUT"
    # the launch stops within a phase of the limit instead of running on
    assert t_cut < 0.5 * t_full
    with pytest.raises(csl.CSLError, match="ERR_TIMEOUT"):
        csl.minres_solve(p, f, timeout_ms=1)
    # the next solve starts clean and repeats the earlier result bitwise
    z_again, info_again = csl.minres_solve(p, f, timeout_ms=30000)
    assert info_again == info_full
    assert torch.equal(z_again, z_full)
    p.close()


def test_time_limit_batch(csl):
    n = 127
    big = (_coef((n, n, n), 9, 1.0, 3.0), complex(10.0, 100.0), _crand((n, n, n), 10))
    small = [(_coef((15, 15), 11 + j), complex(-20.0 + j, 2.0), _crand((15, 15), 20 + j))
             for j in range(4)]
    systems = [big] + small
    probs = [csl.Problem(cuda(a), lam.real, lam.imag, dst="fft") for a, lam, _ in systems]
    fs = [cuda(f) for *_, f in systems]
    # 15 ms: half of the big system's solve (32 ms alone) and several times
    # what the small ones need (2 to 3 ms), so both outcomes occur in one launch
    b_cut = csl.Batch(probs, timeout_ms=15)
    for rep in range(2):
        zs, infos = b_cut.solve(fs, raise_on_error=False)
        _say("limited batch, replay", rep, [(i["status_name"], i["iters"]) for i in infos])
        assert infos[0]["status_name"] == "ERR_TIMEOUT"
        assert any(i["status"] == 0 for i in infos[1:])
        for (a, lam, f), p, z, info in zip(systems[1:], probs[1:], zs[1:], infos[1:]):
            assert info["status_name"] in ("OK", "ERR_TIMEOUT")
            if info["status"] == 0:
                # a system that finished before the limit keeps its solution
                po = O.Problem(a, lam.real, lam.imag)
                zo, io = po.solve(f)
                assert _vs_oracle(po, lam, f, z.cpu().numpy(), info, zo, io) <= 1e-9
    with pytest.raises(csl.CSLError, match="ERR_TIMEOUT"):
        b_cut.solve(fs)
    b_cut.close()
    # a batch of the same problems with room to finish converges everywhere
    b = csl.Batch(probs, timeout_ms=30000)
    zs, infos = b.solve(fs)
    assert all(i["status"] == 0 and i["relres_true"] <= 1e-8 for i in infos), infos
    b.close()
    for p in probs:
        p.close()


def test_batch_rejects_shared_vectors(csl):
    shape = (15, 15)
    probs = [csl.Problem(cuda(_coef(shape, 30 + j)), 5.0 + j, 2.0, dst="fft") for j in range(3)]
    fs = [cuda(_crand(shape, 40 + j)) for j in range(3)]
    zs = [torch.empty_like(f) for f in fs]
    b = csl.Batch(probs, timeout_ms=30000)
    for bad_z in ([zs[0], zs[0], zs[2]],      # two systems, one solution vector
                  [zs[0], fs[0], zs[2]],      # a solution vector is another system's f
                  [fs[0], zs[1], zs[2]]):     # f and z of one system alias
        with pytest.raises(csl.CSLError, match="ERR_ARG"):
            b.solve(fs, zs=bad_z)
    out, infos = b.solve(fs, zs=zs)
    assert all(i["status"] == 0 for i in infos)
    b.close()
    for p in probs:
        p.close()


def test_option_and_alias_checks(csl):
    import ctypes
    from paper_2408_00488_amd import _ptr, _stream
    shape = (15, 15)
    p = csl.Problem(cuda(_coef(shape, 50)), 5.0, 2.0, dst="fft")
    f = cuda(_crand(shape, 51))
    z, _ = csl.minres_solve(p, f)
    L = csl.load_library()
    # the adjoint's gradient in f must not overwrite the forward solution
    st = L.minres_adjoint(p.handle, _ptr(z), _ptr(f), _ptr(z), None, None, None, None, None,
                          _stream(p.device))
    assert st == 1 and "alias" in L.csl_last_error().decode()
    for bad in (dict(tol=float("nan")), dict(maxit=20000000)):
        with pytest.raises(csl.CSLError, match="ERR_ARG"):
            csl.minres_solve(p, f, **bad)
        with pytest.raises(csl.CSLError, match="ERR_ARG"):
            csl.minres_adjoint(p, z, f, **bad)
        with pytest.raises(csl.CSLError, match="ERR_ARG"):
            csl.Batch([p], **bad)
    with pytest.raises(csl.CSLError, match="ERR_ARG"):
        csl.Batch([p], grid_size=-1)
    # nothing above changed the problem: the solve repeats bitwise
    z2, _ = csl.minres_solve(p, f)
    assert torch.equal(z, z2)
    p.close()


def test_problems_from_several_threads(csl):
    # ctypes releases the GIL: four threads create problems and solve on
    # streams of their own at the same time; every result equals the same
    # solve done alone
    import threading
    shapes = [(31, 31), (63, 63), (15, 31, 15), (20, 45)]
    data = [(_coef(s, 60 + j), _crand(s, 70 + j)) for j, s in enumerate(shapes)]
    ref = []
    for a, f in data:
        p = csl.Problem(cuda(a), 8.0, 30.0)
        z, info = csl.minres_solve(p, cuda(f))
        ref.append((z.cpu(), info))
        p.close()
    out = [None] * len(data)
    errors = []

    def work(j):
        try:
            s = torch.cuda.Stream()
            with torch.cuda.stream(s):
                a, f = data[j]
                p = csl.Problem(cuda(a), 8.0, 30.0)
                z, info = csl.minres_solve(p, cuda(f))
                out[j] = (z.cpu(), info)
                p.close()
        except Exception as e:   # reported below
            errors.append((j, repr(e)))

    threads = [threading.Thread(target=work, args=(j,)) for j in range(len(data))]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    assert not errors, errors
    for (zr, ir), (z, i) in zip(ref, out):
        assert i == ir and torch.equal(z, zr)


def test_concurrent_whole_gpu_solves(csl):
    # two single solves on the plane schedule (one 1024-thread workgroup per
    # CU, 254 workgroups each) launched on two streams at once: the second
    # kernel can start only part of its grid while the first runs, so its
    # phases must go to whichever workgroups are resident (tiles are owned
    # by workgroups only once the whole grid has started).  Both finish, and
    # each result equals the same solve run alone, bit for bit.
    shape = (127, 127, 127)
    a = cuda(_coef(shape, 11, 1.0, 3.0))
    fs = [cuda(_crand(shape, 12 + j)) for j in range(2)]
    probs = [csl.Problem(a, 10.0 + 20.0 * j, 100.0, pinv_fp32=True, dst="fft") for j in range(2)]
    for p in probs:
        p.set_schedule(8128, 65536, 1024)
    ref = []
    for p, f in zip(probs, fs):
        z, info = csl.minres_solve(p, f, timeout_ms=30000)
        assert info["status"] == 0, info
        ref.append((z.clone(), info))
    streams = [torch.cuda.Stream() for _ in probs]
    zs = [torch.empty_like(f) for f in fs]
    torch.cuda.synchronize()
    for p, f, z, st in zip(probs, fs, zs, streams):
        with torch.cuda.stream(st):
            csl.minres_solve(p, f, z, timeout_ms=30000, want_info=False)
    torch.cuda.synchronize()
    for z, (zr, ir) in zip(zs, ref):
        _say("concurrent solve", ir["iters"], "iterations alone; equal:", torch.equal(z, zr))
        assert torch.equal(z, zr)
    for p in probs:
        p.close()


@pytest.mark.parametrize("threads,fp32", [(1024, True), (512, False)])
def test_owned_and_claimed_tiles(csl, threads, fp32):
    # one LDS chunk per tile on a 127^3 grid: the row phases have about a
    # thousand tiles for 254 or 512 workgroups, so each phase starts with
    # the tiles the workgroups own and goes on with claimed ones.  The solve
    # converges and agrees with the usual schedule's (1e-6 with the FP32
    # preconditioner, 1e-10 in FP64).
    shape = (127, 127, 127)
    a = cuda(_coef(shape, 21, 1.0, 3.0))
    f = cuda(_crand(shape, 22))
    p = csl.Problem(a, 10.0, 100.0, pinv_fp32=fp32, dst="fft")
    p.set_schedule(8128 if threads == 1024 else 8192, 65536, threads)
    z0, i0 = csl.minres_solve(p, f, timeout_ms=30000)
    p.set_schedule(1, 65536, threads)
    z1, i1 = csl.minres_solve(p, f, timeout_ms=30000)
    _say("owned and claimed", threads, p.schedule["grid_size"], i0["iters"], i1["iters"],
         rel(z1.cpu().numpy(), z0.cpu().numpy()))
    assert i1["status"] == 0 and i1["relres_true"] <= 1e-8
    assert rel(z1.cpu().numpy(), z0.cpu().numpy()) <= (1e-6 if fp32 else 1e-10)
    p.close()


def test_chunk_size_schedule(csl):
    # small grids may run their own solves on 512- or 1024-element chunks;
    # a chunking with more tiles than partial-sum slots is refused and the
    # schedule in force stays
    shape, lam = (63, 63), complex(12.0, 30.0)
    a = _coef(shape, 80)
    f = _crand(shape, 81)
    p = csl.Problem(cuda(a), lam.real, lam.imag)
    po = O.Problem(a, lam.real, lam.imag)
    zo, io = po.solve(f)
    for te in (512, 1024, 0):
        p.set_schedule(0, 0, 0, te)
        assert p.schedule["tile_elems"] == te
        z, info = csl.minres_solve(p, cuda(f))
        assert info["status"] == 0
        assert _vs_oracle(po, lam, f, z.cpu().numpy(), info, zo, io) <= 1e-10
    p.set_schedule(0, 0, 0, 512)
    before = p.schedule
    with pytest.raises(csl.CSLError, match="ERR_ARG"):
        p.set_schedule(0, 0, 0, 16)
    assert p.schedule == before
    p.close()
    big = csl.Problem(cuda(_coef((511, 511), 82)), 1.0, 1.0)
    with pytest.raises(csl.CSLError, match="ERR_ARG"):
        big.set_schedule(0, 0, 0, 512)
    big.close()


def test_batch_isolates_degenerate_systems(csl):
    # a zero right-hand side finishes at step 0, a NaN one with
    # ERR_NONFINITE; the other systems of the same launch converge as alone
    shapes = [(31, 31), (63, 63), (15, 15, 15), (31, 63)]
    probs = [csl.Problem(cuda(_coef(s, 90 + j)), 9.0, 33.0) for j, s in enumerate(shapes)]
    fs_h = [_crand(s, 95 + j) for j, s in enumerate(shapes)]
    fs_h[1] = np.zeros(shapes[1], dtype=np.complex128)
    fs_h[2] = fs_h[2].copy()
    fs_h[2][3, 4, 5] = np.nan
    b = csl.Batch(probs, timeout_ms=30000)
    zs, infos = b.solve([cuda(f) for f in fs_h], raise_on_error=False)
    assert infos[1]["status"] == 0 and infos[1]["iters"] == 0 and not zs[1].abs().sum().item()
    assert infos[2]["status_name"] == "ERR_NONFINITE"
    for j in (0, 3):
        z1, i1 = csl.minres_solve(probs[j], cuda(fs_h[j]))
        assert infos[j]["status"] == 0 and abs(infos[j]["iters"] - i1["iters"]) <= 1
        assert float((zs[j] - z1).abs().max() / z1.abs().max()) <= 1e-9
    with pytest.raises(csl.CSLError, match="ERR_NONFINITE"):
        b.solve([cuda(f) for f in fs_h])
    b.close()
    for p in probs:
        p.close()
