"""The C-ABI library on the host: it loads without a GPU, exports every
function include/lpsift.h declares, and rejects bad arguments with a status
code before any GPU call (no pointer passed here is ever dereferenced)."""
import ctypes
import math
import os
import re

import pytest

import paper_2405_08578_amd as lp
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FAKE = 0x10000          # a non-null "device" address that validation never touches


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(lp.LIB_PATH):
        from paper_2405_08578_amd import build
        build.build()
    return lp.load()


def declared_functions():
    txt = open(os.path.join(ROOT, "include", "lpsift.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(lpsift_[a-z0-9_]+)\s*\(", txt)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert len(names) >= 8
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(lp.EXPORTS)


def test_version_and_status_strings(lib):
    assert lib.lpsift_version() >= 100
    for st in (0, -1, -2, -3, -4):
        assert lp.status_string(st) != "unknown status"
    assert lp.status_string(7) == "unknown status"


@pytest.mark.parametrize("h,w,Ls", [(480, 640, [16, 32, 64]), (1600, 2600, [16, 32, 64, 128]),
                                    (1, 1, [4]), (33, 97, [4, 8, 24])])
def test_num_keypoints_matches_oracle(lib, h, w, Ls):
    assert lp.num_keypoints(h, w, lp.Params(Ls)) == oracle.num_keypoints(h, w, Ls)


def test_num_keypoints_rejects(lib):
    p = lp.Params([16])
    assert lib.lpsift_num_keypoints(0, 10, ctypes.byref(p.c())) == -1
    assert lib.lpsift_num_keypoints(10, 10, None) == -1


def image(h=64, w=64, pitch=None):
    im = lp.lpsift_image()
    im.data, im.height, im.width = FAKE, h, w
    im.pitch = w if pitch is None else pitch
    return im


def kps(n):
    k = lp.lpsift_keypoints()
    for f in ("x", "y", "scale", "type", "value", "contrast"):
        setattr(k, f, FAKE)
    k.capacity = n
    return k


def detect(lib, params, ims, ks):
    a = (lp.lpsift_image * len(ims))(*ims)
    b = (lp.lpsift_keypoints * len(ks))(*ks)
    return lib.lpsift_detect(a, len(ims), ctypes.byref(params), b, None)


def test_detect_validation(lib):
    P = lp.Params([16, 32]).c()
    n = lp.num_keypoints(64, 64, lp.Params([16, 32]))
    assert detect(lib, P, [image(pitch=10)], [kps(n)]) == lp.LPSIFT_EINVAL
    assert detect(lib, P, [image(h=0)], [kps(n)]) == lp.LPSIFT_EINVAL
    assert detect(lib, P, [image()], [kps(n - 1)]) == lp.LPSIFT_ECAPACITY
    k = kps(n)
    k.contrast = None
    assert detect(lib, P, [image()], [k]) == lp.LPSIFT_EINVAL
    im = image()
    im.data = None
    assert detect(lib, P, [im], [kps(n)]) == lp.LPSIFT_EINVAL
    bad = lp.Params([32, 16]).c()                       # not ascending
    assert detect(lib, bad, [image()], [kps(10**6)]) == lp.LPSIFT_EINVAL
    small = lp.Params([2, 16]).c()                      # L below 4
    assert detect(lib, small, [image()], [kps(10**6)]) == lp.LPSIFT_EINVAL
    huge = lp.Params([16, 70000]).c()                   # L above 65536
    assert detect(lib, huge, [image()], [kps(10**6)]) == lp.LPSIFT_EINVAL
    nonnested = lp.Params([32, 40]).c()                 # any set is valid: capacity checked
    nk = lp.num_keypoints(64, 64, lp.Params([32, 40]))
    assert detect(lib, nonnested, [image()], [kps(nk - 1)]) == lp.LPSIFT_ECAPACITY
    d8 = lp.Params([16, 32], d=8).c()
    assert detect(lib, d8, [image()], [kps(10**6)]) == lp.LPSIFT_EUNSUPPORTED
    zero = lp.lpsift_params()
    assert detect(lib, zero, [image()], [kps(n)]) == lp.LPSIFT_EINVAL
    a = (lp.lpsift_image * 1)(image())
    assert lib.lpsift_detect(a, 0, ctypes.byref(P), (lp.lpsift_keypoints * 1)(kps(n)), None) \
        == lp.LPSIFT_EINVAL


def test_describe_validation_and_workspace(lib):
    prm = lp.Params([16, 32, 64, 128])
    P = prm.c()
    ims = (lp.lpsift_image * 2)(image(1600, 2600), image(480, 640))
    need = lib.lpsift_describe_workspace_size(ims, 2, ctypes.byref(P))
    # the two gradient fields (8 bytes per pixel) and the disc tables: 16 bytes
    # per entry, each descriptor disc once per orientation bucket (64 x at most
    # the 9,436 entries of the four discs at L = 16..128)
    assert need >= 8 * (1600 * 2600 + 480 * 640)
    assert need < 8 * (1600 * 2600 + 480 * 640) + 16 * (64 * 9436 + 2000) + (1 << 16)
    n0 = lp.num_keypoints(1600, 2600, prm)
    n1 = lp.num_keypoints(480, 640, prm)
    ks = (lp.lpsift_keypoints * 2)(kps(n0), kps(n1))
    th = (ctypes.c_void_p * 2)(FAKE, FAKE)
    de = (ctypes.c_void_p * 2)(FAKE, FAKE)
    ws = 0x100000
    call = lambda wsb, k=ks, t=th: lib.lpsift_describe(ims, 2, k, ctypes.byref(P), ws, wsb, t, de, None)
    assert call(need - 1) == lp.LPSIFT_ECAPACITY
    ks2 = (lp.lpsift_keypoints * 2)(kps(n0), kps(n1 - 1))
    assert call(need, k=ks2) == lp.LPSIFT_ECAPACITY
    th2 = (ctypes.c_void_p * 2)(FAKE, None)
    assert call(need, t=th2) == lp.LPSIFT_EINVAL
    assert lib.lpsift_describe(ims, 2, ks, ctypes.byref(P), ws + 4, need, th, de, None) \
        == lp.LPSIFT_EINVAL                              # workspace not 256-byte aligned


def test_match_validation_and_workspace(lib):
    mp = lp.match_params()
    nA, nB = [43396], [43396]
    need = lp.match_workspace_size(nA, nB, mp)
    assert need >= 4 * 43396
    arr = lambda *v: (ctypes.c_void_p * len(v))(*v)
    i64 = lambda *v: (ctypes.c_int64 * len(v))(*v)

    def call(mp_, nA_=43396, nB_=43396, ws=0x100000, wsb=need, dA=FAKE):
        return lib.lpsift_match(arr(dA), i64(nA_), arr(FAKE), i64(nB_), 1, ctypes.byref(mp_), ws,
                                wsb, arr(FAKE), arr(FAKE), arr(FAKE), None)
    assert call(mp, wsb=need - 1) == lp.LPSIFT_ECAPACITY
    assert call(mp, nA_=-1) == lp.LPSIFT_EINVAL
    assert call(mp, dA=FAKE + 4) == lp.LPSIFT_EINVAL         # not 16-byte aligned
    assert call(mp, ws=0x100000 + 8) == lp.LPSIFT_EINVAL
    for bad in (lp.match_params(ratio=0.0), lp.match_params(ratio=math.nan),
                lp.match_params(ratio=-math.inf),
                lp.match_params(abs_thresh=math.nan), lp.match_params(abs_thresh=-1.0),
                lp.match_params(b_chunks=17), lp.match_params(precision=4),
                lp.match_params(qblock_waves=3), lp.match_params(qblock_waves=16),
                lp.match_params(qblock_waves=-1),
                # topk: 2 .. 8 at precisions 1 and 2 only
                lp.match_params(precision=1, topk=1), lp.match_params(precision=2, topk=9),
                lp.match_params(precision=1, topk=-1), lp.match_params(precision=0, topk=2),
                lp.match_params(precision=3, topk=8)):
        assert call(bad) == lp.LPSIFT_EINVAL
    for prec in (1, 2):
        for k in (2, 5, 8):   # accepted: the workspace check comes next
            assert call(lp.match_params(precision=prec, topk=k)) == lp.LPSIFT_ECAPACITY
    for w in (2, 4, 8):
        assert lp.match_workspace_size(nA, nB, lp.match_params(qblock_waves=w)) > 0
    # low-precision paths need more workspace (quantised copies, keys, FP32 fallback)
    for prec in (1, 2, 3):
        mlp = lp.match_params(precision=prec)
        assert lp.match_workspace_size(nA, nB, mlp) > need
        assert call(mlp) == lp.LPSIFT_ECAPACITY
    assert lp.match_workspace_size([10], [0], mp) >= 0


def test_match_noalloc_validation(lib):
    """The fixed scratch size in the binding equals the header's, and calls
    whose workspace need exceeds it are rejected before any GPU work."""
    txt = open(os.path.join(ROOT, "include", "lpsift.h")).read()
    m = re.search(r"#define LPSIFT_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", txt)
    assert m and int(m.group(1)) << int(m.group(2)) == lp.NOALLOC_SCRATCH_BYTES
    arr = lambda *v: (ctypes.c_void_p * len(v))(*v)
    i64 = lambda *v: (ctypes.c_int64 * len(v))(*v)

    def call(mp_, n=43396, dA=FAKE):
        return lib.lpsift_match_noalloc(arr(dA), i64(n), arr(FAKE), i64(n), 1, ctypes.byref(mp_),
                                        arr(FAKE), arr(FAKE), arr(FAKE), None)
    m3 = lp.match_params(precision=3)
    assert lp.match_workspace_size([43396], [43396], m3) > lp.NOALLOC_SCRATCH_BYTES
    assert call(m3) == lp.LPSIFT_ECAPACITY
    for prec in (0, 1, 2):      # these fit at 43,396 x 43,396
        assert lp.match_workspace_size([43396], [43396], lp.match_params(precision=prec)) \
            <= lp.NOALLOC_SCRATCH_BYTES
    assert call(lp.match_params(), n=-1) == lp.LPSIFT_EINVAL
    assert call(lp.match_params(), dA=FAKE + 4) == lp.LPSIFT_EINVAL
    assert call(lp.match_params(ratio=0.0)) == lp.LPSIFT_EINVAL
    assert call(lp.match_params(precision=4)) == lp.LPSIFT_EINVAL


def test_match_tune_validation(lib):
    mp = lp.match_params()
    nA, nB = [5000, 300], [4000, 0]
    arr = lambda *v: (ctypes.c_void_p * len(v))(*v)
    i64 = lambda *v: (ctypes.c_int64 * len(v))(*v)
    needs = []
    for c in (1, 16):
        m = lp.match_params(b_chunks=c)
        needs.append(lp.match_workspace_size(nA, nB, m))
    assert needs[1] > needs[0]             # more chunks keep more candidates per query
    ms = (ctypes.c_float * 16)()
    best = ctypes.c_int32(0)
    best_w = ctypes.c_int32(0)

    def call(cands, reps=2, wsb=max(needs), m=mp, msp=ms, bp=ctypes.byref(best), dA=FAKE,
             waves=(), wp=ctypes.byref(best_w)):
        k = len(cands)
        nw = len(waves) if waves is not None else 1
        wa = (ctypes.c_int32 * max(nw, 1))(*waves) if waves is not None else None
        return lib.lpsift_match_tune(arr(dA, FAKE), i64(*nA), arr(FAKE, FAKE), i64(*nB), 2,
                                     ctypes.byref(m), (ctypes.c_int32 * max(k, 1))(*cands), k,
                                     wa, nw, reps, 0x100000, wsb,
                                     arr(FAKE, FAKE), arr(FAKE, FAKE), arr(FAKE, FAKE), msp, bp,
                                     wp, None)
    assert call([1, 16], wsb=needs[1] - 1) == lp.LPSIFT_ECAPACITY   # the largest must fit
    assert call([0, 4]) == lp.LPSIFT_EINVAL
    assert call([17]) == lp.LPSIFT_EINVAL
    assert call([]) == lp.LPSIFT_EINVAL
    assert call([2], reps=0) == lp.LPSIFT_EINVAL
    assert call([2], msp=None) == lp.LPSIFT_EINVAL
    assert call([2], bp=None) == lp.LPSIFT_EINVAL
    assert call([2], dA=FAKE + 4) == lp.LPSIFT_EINVAL
    assert call([2], m=lp.match_params(ratio=-1.0)) == lp.LPSIFT_EINVAL
    # the wave-count dimension: each value 0, 2, 4 or 8, arrays given when used
    assert call([2], waves=(3,)) == lp.LPSIFT_EINVAL
    assert call([2], waves=(2, 16)) == lp.LPSIFT_EINVAL
    assert call([2], waves=None) == lp.LPSIFT_EINVAL            # n_waves 1, no array
    assert call([2], waves=(2, 4), wp=None) == lp.LPSIFT_EINVAL
    assert call([2], m=lp.match_params(qblock_waves=5)) == lp.LPSIFT_EINVAL


def test_tune_bucket():
    assert [lp._bucket(n) for n in (0, 1, 2, 3, 1000, 1024, 1025)] == [0, 1, 2, 4, 1024, 1024, 2048]


def test_timing_ids_and_validation(lib):
    txt = open(os.path.join(ROOT, "include", "lpsift.h")).read()
    ids = dict((m.group(1).lower(), int(m.group(2)))
               for m in re.finditer(r"LPSIFT_KERNEL_([A-Z0-9_]+)\s*=\s*(\d+)", txt))
    count = ids.pop("count")
    assert len(lp.KERNELS) == count == len(ids)
    for name, k in ids.items():
        assert lp.KERNELS[k] == name
    ms, n = ctypes.c_double(0), ctypes.c_int64(0)
    assert lib.lpsift_timing_read(count, ctypes.byref(ms), ctypes.byref(n)) == lp.LPSIFT_EINVAL
    assert lib.lpsift_timing_read(-1, ctypes.byref(ms), ctypes.byref(n)) == lp.LPSIFT_EINVAL
    assert lib.lpsift_timing_read(0, None, ctypes.byref(n)) == lp.LPSIFT_EINVAL
    lp.timing_enable(True)
    t = lp.timing_read()            # nothing launched: no HIP call is needed
    assert all(v["launches"] == 0 and v["ms"] == 0.0 for v in t.values())
    lp.timing_enable(False)


def test_scorer_entry_validation(lib):
    P = lp.Params([16, 32]).c()
    n = lp.num_keypoints(64, 64, lp.Params([16, 32]))
    ims = (lp.lpsift_image * 1)(image())
    ks = (lp.lpsift_keypoints * 1)(kps(n))
    arr = lambda *v: (ctypes.c_void_p * len(v))(*v)
    i64 = lambda *v: (ctypes.c_int64 * len(v))(*v)
    # score
    assert lib.lpsift_score(ims, 1, ks, ctypes.byref(P), None, arr(FAKE), None) == lp.LPSIFT_EINVAL
    assert lib.lpsift_score(ims, 1, ks, ctypes.byref(P), FAKE, arr(None), None) == lp.LPSIFT_EINVAL
    small = (lp.lpsift_keypoints * 1)(kps(n - 1))
    assert lib.lpsift_score(ims, 1, small, ctypes.byref(P), FAKE, arr(FAKE), None) \
        == lp.LPSIFT_ECAPACITY
    # prune: k <= n, non-negative, pointers
    assert lib.lpsift_prune(arr(FAKE), i64(10), i64(11), 1, arr(FAKE), None) == lp.LPSIFT_EINVAL
    assert lib.lpsift_prune(arr(FAKE), i64(-1), i64(0), 1, arr(FAKE), None) == lp.LPSIFT_EINVAL
    assert lib.lpsift_prune(arr(None), i64(10), i64(3), 1, arr(FAKE), None) == lp.LPSIFT_EINVAL
    assert lib.lpsift_prune(arr(FAKE), i64(10), i64(3), 1, arr(None), None) == lp.LPSIFT_EINVAL
    assert lib.lpsift_prune(arr(FAKE), i64(10), i64(3), 0, arr(FAKE), None) == lp.LPSIFT_EINVAL
    assert lib.lpsift_prune(arr(FAKE + 4), i64(10), i64(3), 1, arr(FAKE), None) == lp.LPSIFT_EINVAL
    # describe_selected
    ws = 0x100000
    need = lib.lpsift_describe_workspace_size(ims, 1, ctypes.byref(P))
    call = lambda sel, ns, wsb=need: lib.lpsift_describe_selected(
        ims, 1, ks, ctypes.byref(P), sel, ns, ws, wsb, arr(FAKE), arr(FAKE), None)
    assert call(arr(FAKE), i64(-1)) == lp.LPSIFT_EINVAL
    assert call(arr(None), i64(5)) == lp.LPSIFT_EINVAL
    assert call(None, i64(5)) == lp.LPSIFT_EINVAL
    assert call(arr(FAKE), i64(5), need - 1) == lp.LPSIFT_ECAPACITY
    # gather: 4-byte aligned patches
    assert lib.lpsift_scorer_gather(ims, 1, ks, ctypes.byref(P), None, None, arr(FAKE + 1),
                                    arr(FAKE), None) == lp.LPSIFT_EINVAL
    assert lib.lpsift_scorer_gather(ims, 1, ks, ctypes.byref(P), arr(FAKE), None, arr(FAKE),
                                    arr(FAKE), None) == lp.LPSIFT_EINVAL
    # training step
    assert lib.lpsift_scorer_train_workspace_size(0) == 0
    wsz = lib.lpsift_scorer_train_workspace_size(100)
    assert wsz >= 2 * (20801 + 2) * 4                  # two partial-sum rows of 64 candidates
    step = lambda b=100, t=1, lr=1e-3, wsb=wsz: lib.lpsift_scorer_train_step(
        FAKE, FAKE, FAKE, FAKE, b, FAKE, FAKE, FAKE, t, lr, ws, wsb, None, None)
    assert step(b=0) == lp.LPSIFT_EINVAL
    assert step(t=0) == lp.LPSIFT_EINVAL
    assert step(lr=0.0) == lp.LPSIFT_EINVAL
    assert step(lr=math.nan) == lp.LPSIFT_EINVAL
    assert step(wsb=wsz - 1) == lp.LPSIFT_ECAPACITY


def test_ransac_gpu_validation(lib):
    arr = lambda *v: (ctypes.c_void_p * len(v))(*v)
    i64 = lambda *v: (ctypes.c_int64 * len(v))(*v)
    k = (lp.lpsift_keypoints * 1)(kps(100))
    need = lib.lpsift_ransac_workspace_size(i64(1000), 1, 2000)
    assert need > 2 * 1000 * 16
    assert lib.lpsift_ransac_workspace_size(i64(-1), 1, 10) == 0
    assert lib.lpsift_ransac_workspace_size(i64(10), 1, (1 << 20) + 1) == 0

    def call(n_iter=2000, tries=8, thresh=3.0, u=FAKE, wsb=need, ws=0x100000, nq=1000):
        rp = lp.lpsift_ransac_params(n_iter, tries, thresh, u)
        return lib.lpsift_ransac(k, k, None, None, arr(FAKE), i64(nq), 1, ctypes.byref(rp), ws, wsb,
                                 arr(FAKE), arr(FAKE), arr(FAKE), FAKE, FAKE, None)
    assert call(wsb=need - 1) == lp.LPSIFT_ECAPACITY
    assert call(tries=0) == lp.LPSIFT_EINVAL
    assert call(tries=65) == lp.LPSIFT_EINVAL
    assert call(thresh=0.0) == lp.LPSIFT_EINVAL
    assert call(thresh=math.inf) == lp.LPSIFT_EINVAL
    assert call(u=None) == lp.LPSIFT_EINVAL
    assert call(n_iter=-1) == lp.LPSIFT_EINVAL
    assert call(ws=0x100000 + 8) == lp.LPSIFT_EINVAL
    assert call(nq=-5) == lp.LPSIFT_EINVAL


def test_quantize_lowp_validation(lib):
    A = ctypes.c_void_p(1 << 20)                 # never dereferenced: every call below fails first
    S = ctypes.c_void_p(1 << 22)
    E = lp.LPSIFT_EINVAL
    q = lib.lpsift_quantize_lowp
    assert q(A, 4, 0, A, S, None) == E                              # bad precision
    assert q(A, 4, 3, A, S, None) == E
    assert q(A, -1, 1, A, None, None) == E
    assert q(None, 4, 1, A, None, None) == E
    assert q(A, 4, 2, A, None, None) == E                           # FP8 needs scales
    assert q(ctypes.c_void_p((1 << 20) + 4), 4, 1, A, None, None) == E
    assert q(A, 4, 1, ctypes.c_void_p((1 << 20) + 8), None, None) == E   # BF16 rows: 16 B
    assert q(A, 4, 2, ctypes.c_void_p((1 << 20) + 4), S, None) == E      # FP8 rows: 8 B
    assert q(A, 4, 2, A, ctypes.c_void_p((1 << 22) + 2), None) == E
    assert q(None, 0, 1, None, None, None) == lp.LPSIFT_OK           # nothing to do


def test_u8_entry_validation(lib):
    A = ctypes.c_void_p(1 << 20)                 # never dereferenced: every call below fails first
    ws = ctypes.c_void_p(1 << 21)
    E = lp.LPSIFT_EINVAL
    assert lib.lpsift_quantize_u8(None, 3, A, None) == E
    assert lib.lpsift_quantize_u8(A, -1, A, None) == E
    assert lib.lpsift_quantize_u8(ctypes.c_void_p((1 << 20) + 4), 1, A, None) == E
    assert lib.lpsift_quantize_u8(A, 1, ctypes.c_void_p((1 << 20) + 2), None) == E
    assert lib.lpsift_quantize_u8(None, 0, None, None) == lp.LPSIFT_OK    # nothing to do
    assert lib.lpsift_match_u8_workspace_size(-1, 5) == 0
    assert lib.lpsift_match_u8_workspace_size(5, 1 << 31) == 0
    small = lib.lpsift_match_u8_workspace_size(100, 300)
    big = lib.lpsift_match_u8_workspace_size(60000, 60000)
    assert 0 < small < big

    def call(qA=A, nA=10, qB=A, nB=10, ratio=0.8, thr=math.inf, w=ws, nbytes=1 << 30, out=A):
        return lib.lpsift_match_u8(qA, nA, qB, nB, ratio, thr, w, nbytes, out, out, out, None)
    assert call(nA=-1) == E
    assert call(nB=1 << 31) == E
    assert call(ratio=0.0) == E
    assert call(ratio=math.nan) == E
    assert call(thr=math.nan) == E
    assert call(thr=0.0) == E
    assert call(qA=None) == E
    assert call(qB=None) == E
    assert call(out=None) == E
    assert call(qA=ctypes.c_void_p((1 << 20) + 8)) == E
    assert call(w=ctypes.c_void_p((1 << 21) + 64)) == E
    assert call(w=None) == E
    assert call(nbytes=lib.lpsift_match_u8_workspace_size(10, 10) - 1) == lp.LPSIFT_ECAPACITY
    assert call(nA=0, qA=None, out=None) == lp.LPSIFT_OK                   # no queries: no launch


def test_describe_multi_validation(lib):
    P = lp.Params([16, 32]).c()
    im = lp.lpsift_image()
    im.data, im.height, im.width, im.pitch = 1 << 20, 64, 64, 64
    ims = (lp.lpsift_image * 1)(im)
    n_kp = lp.num_keypoints(64, 64, lp.Params([16, 32]))
    kp = lp.lpsift_keypoints()
    kp.x = kp.y = kp.scale = kp.type = kp.value = kp.contrast = 1 << 22
    kp.capacity = n_kp
    kps = (lp.lpsift_keypoints * 1)(kp)
    need = lib.lpsift_describe_multi_workspace_size(ims, 1, ctypes.byref(P))
    assert need > lib.lpsift_describe_workspace_size(ims, 1, ctypes.byref(P))
    buf = (ctypes.c_void_p * 1)(1 << 23)
    E = lp.LPSIFT_EINVAL

    def call(mo=4, pr=0.8, ws=1 << 24, nbytes=need, rows=buf, n_rows=1 << 25):
        return lib.lpsift_describe_multi(ims, 1, kps, ctypes.byref(P), mo, pr, ws, nbytes, rows,
                                         buf, buf, n_rows, None)
    assert call(mo=0) == E
    assert call(mo=5) == E
    assert call(pr=0.0) == E
    assert call(pr=1.5) == E
    assert call(pr=math.nan) == E
    assert call(rows=None) == E
    assert call(n_rows=None) == E
    assert call(n_rows=(1 << 25) + 4) == E
    assert call(ws=(1 << 24) + 128) == E
    assert call(nbytes=need - 1) == lp.LPSIFT_ECAPACITY


def test_warp_blend_validation(lib):
    import numpy as np
    im = lp.lpsift_image()
    im.data, im.height, im.width, im.pitch = 1 << 20, 30, 40, 40
    ims = (lp.lpsift_image * 2)(im, im)
    G = np.tile(np.eye(3).reshape(1, 9), (2, 1))
    E = lp.LPSIFT_EINVAL
    cv = ctypes.c_void_p(1 << 22)

    def call(n=2, g=G, w=50, h=40, canvas=cv, x0=0.0):
        g = np.ascontiguousarray(g, np.float64)
        return lib.lpsift_warp_blend(ims, n, g.ctypes.data, x0, 0.0, w, h, canvas, None, None)
    assert call(n=0) == E
    assert call(n=17) == E
    assert lib.lpsift_warp_blend(ims, 2, None, 0.0, 0.0, 5, 5, cv, None, None) == E
    bad = G.copy()
    bad[1, 4] = np.nan
    assert call(g=bad) == E
    sing = G.copy()
    sing[0] = [1, 2, 0, 2, 4, 0, 0, 0, 1]           # rank 2
    assert call(g=sing) == E
    assert call(w=-1) == E
    assert call(w=1 << 16, h=1 << 16) == E
    assert call(canvas=None) == E
    assert call(x0=math.inf) == E
    assert call(w=0, h=0, canvas=None) == lp.LPSIFT_OK        # empty canvas: nothing launched


def test_mosaic_canvas_bounds_matches_oracle():
    import numpy as np
    from paper_2405_08578_amd import mosaic
    from oracle import warp as W
    rng = np.random.default_rng(0)
    for _ in range(20):
        shapes = [(int(rng.integers(5, 300)), int(rng.integers(5, 300))) for _ in range(3)]
        G = []
        for _ in shapes:
            g = np.eye(3)
            g[:2, :2] += rng.normal(0, 0.2, (2, 2))
            g[:2, 2] = rng.uniform(-500, 500, 2)
            g[2, :2] = rng.normal(0, 1e-4, 2)
            G.append(g)
        assert mosaic.canvas_bounds(shapes, G) == W.canvas_bounds(shapes, G)


def test_probe_validation(lib):
    out = ctypes.c_void_p(1 << 20)
    assert lib.lpsift_probe_out_size() == 2048 * 4
    assert lib.lpsift_probe(4, 10, out, None) == lp.LPSIFT_EINVAL
    assert lib.lpsift_probe(-1, 10, out, None) == lp.LPSIFT_EINVAL
    assert lib.lpsift_probe(0, 0, out, None) == lp.LPSIFT_EINVAL
    assert lib.lpsift_probe(0, (1 << 24) + 1, out, None) == lp.LPSIFT_EINVAL
    assert lib.lpsift_probe(0, 10, None, None) == lp.LPSIFT_EINVAL
    # 2 x 32 x 32 x K multiply-adds per MFMA, 4 chains, one per wavefront
    waves = 2048 * 4
    assert lib.lpsift_probe_ops(0, 3) == 2 * 32 * 32 * 2 * 4 * 3 * waves
    assert lib.lpsift_probe_ops(1, 3) == 2 * 32 * 32 * 16 * 4 * 3 * waves
    assert lib.lpsift_probe_ops(2, 3) == 2 * 32 * 32 * 64 * 4 * 3 * waves
    assert lib.lpsift_probe_ops(3, 3) == 2 * 32 * 32 * 32 * 4 * 3 * waves
    assert lib.lpsift_probe_ops(7, 3) == 0.0
