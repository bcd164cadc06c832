"""Plain CPU oracle of the event-based optical-flow hot path (arXiv 2112.10591).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no
code with the GPU library (``paper_2112_10591_amd``) and never imports it.

The arithmetic lives in ``ebof_oracle.c`` (plain C, double precision,
single-threaded, compiled without FMA contraction); this module only loads it
and marshals NumPy arrays.  Each wrapper names the passage of the paper that
its C function follows.

Parity status (what pins each function; the tests under ``tests/`` hold them):
  edge_image        Sec. III-A       pinned: hand-built event lists, golden file
  denoise / fill    Alg. 1 / Alg. 2  pinned: golden worked examples, identities
  edt_separable     Sec. III-C       pinned: brute force (the definition)
  surface           Eq. (1)-(3)      pinned: closed form values, saturation index
  pyr_down          (flow pyramid)   pinned: scipy.ndimage mirror convolution
  dis_flow          Sec. III-D       pinned: zero motion, linear-ramp sub-pixel
                                     shifts, integer shifts, known translation
  densify           (DIS step)       pinned: hand-worked weights (the 255 scale,
                                     the max(1, .)), cover of clamped patches
  dis_level         (DIS step)       pinned: reset threshold, norm and target on
                                     ramps / paraboloid; damped contraction
  patch_init_*      (DIS step)       pinned: hand-worked start points (patch
                                     centre, factor 2; warm start scale)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "ebof_oracle.c")
_SO = os.path.join(_HERE, "_build", "libebof_oracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with the system C compiler; return the .so path."""
    if not force and os.path.exists(_SO):
        return _SO
    os.makedirs(os.path.dirname(_SO), exist_ok=True)
    tmp = _SO + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-std=c99", "-fPIC", "-shared",
           "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_SO):
        build()
    lib = ctypes.CDLL(_SO)
    P = ctypes.c_void_p
    i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    lib.oref_edge_image.argtypes = [i32, i32, P, P, P, i64, i64, i64, P]
    lib.oref_edge_image.restype = i64
    lib.oref_denoise.argtypes = [i32, i32, P, i32, P]
    lib.oref_fill.argtypes = [i32, i32, P, i32, P]
    lib.oref_edt_brute.argtypes = [i32, i32, P, P]
    lib.oref_edt_brute_at.argtypes = [i32, i32, P, i32, i32]
    lib.oref_edt_brute_at.restype = i32
    lib.oref_edt_separable.argtypes = [i32, i32, P, P]
    lib.oref_surface.argtypes = [i64, P, f64, P]
    lib.oref_pyr_down.argtypes = [i32, i32, P, P]
    lib.oref_surface_kind.argtypes = [i64, P, f64, i32, P]
    lib.oref_flow_errors.argtypes = [i64, P, P, P, P, P]
    lib.oref_flow_errors.restype = i64
    lib.oref_fwl.argtypes = [i32, i32, P, P, P, P, i64, i64, i64, P, P, P]
    lib.oref_fwl.restype = f64
    lib.oref_window_end_area.argtypes = [i32, i32, P, P, i64, i64, i32, i32]
    lib.oref_window_end_area.restype = i64
    lib.oref_var_refine.argtypes = [i32, i32, P, P, P, i32, i32, f64, f64, f64, f64]
    lib.oref_dis_flow_refined.argtypes = [i32, i32, i32, P, P, i32, i32, i32, f64, P, P, P, P]
    lib.oref_dis_flow_refined.restype = ctypes.c_int
    lib.oref_dis_flow.argtypes = [i32, i32, i32, P, P, i32, i32, i32, f64, P, P]
    lib.oref_dis_flow.restype = ctypes.c_int
    lib.oref_dis_flow_warm.argtypes = [i32, i32, i32, P, P, i32, i32, i32, f64, P, P, P]
    lib.oref_dis_flow_warm.restype = ctypes.c_int
    lib.oref_patch_init_coarser.argtypes = [i32, i32, i32, i32, P, i32, i32, P]
    lib.oref_patch_init_previous.argtypes = [i32, i32, i32, i32, i32, P, i32, i32, P]
    lib.oref_dis_level.argtypes = [i32, i32, P, P, i32, i32, i32, f64, P, P]
    lib.oref_densify.argtypes = [i32, i32, P, P, i32, i32, P, P]
    lib.oref_patch_count.argtypes = [i32, i32, i32, i32]
    lib.oref_patch_count.restype = i64
    lib.oref_ff_transport.argtypes = [i32, i32, P, P]
    lib.oref_ff_smooth.argtypes = [i32, i32, i32, P]
    lib.oref_flow_filter.argtypes = [i32, i32, i32, P, P, i32, P, P, P, P]
    lib.oref_flow_filter.restype = ctypes.c_int
    _lib = lib
    return lib


def _ptr(a: np.ndarray):
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.c_void_p)


# --------------------------------------------------------------------------
# Section III-A: window selection and the binary edge image
# --------------------------------------------------------------------------
def edge_image(W, H, x, y, t, t0, dt):
    """Edge image of the events with t0 <= t < t0+dt (Sec. III-A); returns
    (E uint8[H,W] of 0/1, number of events not binned)."""
    x = np.ascontiguousarray(x, np.uint16)
    y = np.ascontiguousarray(y, np.uint16)
    t = np.ascontiguousarray(t, np.int64)
    E = np.zeros((H, W), np.uint8)
    dropped = _load().oref_edge_image(W, H, _ptr(x), _ptr(y), _ptr(t), len(x),
                                      int(t0), int(dt), _ptr(E))
    return E, int(dropped)


def denoise(E, n_d):
    """Algorithm 1 (denoising) with threshold N_d."""
    E = np.ascontiguousarray(E, np.uint8)
    H, W = E.shape
    out = np.empty_like(E)
    _load().oref_denoise(W, H, _ptr(E), int(n_d), _ptr(out))
    return out


def fill(Ed, n_f):
    """Algorithm 2 (filling) with threshold N_f."""
    Ed = np.ascontiguousarray(Ed, np.uint8)
    H, W = Ed.shape
    out = np.empty_like(Ed)
    _load().oref_fill(W, H, _ptr(Ed), int(n_f), _ptr(out))
    return out


def denoise_fill(E, n_d, n_f):
    """Denoising then filling, in that order (Sec. III-B)."""
    return fill(denoise(E, n_d), n_f)


# --------------------------------------------------------------------------
# Section III-C: squared Euclidean distance to the closest edge pixel
# --------------------------------------------------------------------------
INT32_MAX = 2**31 - 1


def edt_brute(E):
    E = np.ascontiguousarray(E, np.uint8)
    H, W = E.shape
    D2 = np.empty((H, W), np.int32)
    _load().oref_edt_brute(W, H, _ptr(E), _ptr(D2))
    return D2


def edt_brute_at(E, px, py):
    E = np.ascontiguousarray(E, np.uint8)
    H, W = E.shape
    return int(_load().oref_edt_brute_at(W, H, _ptr(E), int(px), int(py)))


def edt_separable(E):
    E = np.ascontiguousarray(E, np.uint8)
    H, W = E.shape
    D2 = np.empty((H, W), np.int32)
    _load().oref_edt_separable(W, H, _ptr(E), _ptr(D2))
    return D2


def surface(D2, alpha):
    """Equation (1) on squared distances; float32 result."""
    D2 = np.ascontiguousarray(D2, np.int32)
    S = np.empty(D2.shape, np.float32)
    _load().oref_surface(D2.size, _ptr(D2), float(alpha), _ptr(S))
    return S


SURFACE_EXP, SURFACE_LINEAR, SURFACE_BOUNDED, SURFACE_LOG = 0, 1, 2, 3


def surface_kind(D2, alpha, kind):
    """The ablation surfaces of Sec. IV-B on squared distances (float32):
    0 eq. (1), 1 DS_L (d), 2 DS_LB (min(d, alpha ln 255)), 3 DS_Log (ln(d+1))."""
    D2 = np.ascontiguousarray(D2, np.int32)
    S = np.empty(D2.shape, np.float32)
    _load().oref_surface_kind(D2.size, _ptr(D2), float(alpha), int(kind), _ptr(S))
    return S


def flow_errors(u, v, mask=None):
    """(AEE, outlier fraction, pixels counted) of flow u against ground
    truth v ([2, H, W] each) over mask (all pixels when None), Sec. IV."""
    u = np.ascontiguousarray(u, np.float64)
    v = np.ascontiguousarray(v, np.float64)
    m = None if mask is None else np.ascontiguousarray(mask, np.uint8)
    aee, out = ctypes.c_double(), ctypes.c_double()
    n = _load().oref_flow_errors(u[0].size, _ptr(u), _ptr(v), _ptr(m) if m is not None else None,
                                 ctypes.byref(aee), ctypes.byref(out))
    return aee.value, out.value, int(n)


def fwl(W, H, x, y, t, t0, dt, flow, pol=None):
    """Flow warp loss of one window's events under flow ([2, H, W], pixels
    per dt), Sec. IV: (fwl, variance compensated, variance uncompensated)."""
    x = np.ascontiguousarray(x, np.uint16)
    y = np.ascontiguousarray(y, np.uint16)
    t = np.ascontiguousarray(t, np.int64)
    f = np.ascontiguousarray(flow, np.float64)
    pp = None if pol is None else np.ascontiguousarray(pol, np.int8)
    vc, vu = ctypes.c_double(), ctypes.c_double()
    r = _load().oref_fwl(int(W), int(H), _ptr(x), _ptr(y), _ptr(t), _ptr(pp) if pp is not None else None,
                         x.size, int(t0), int(dt), _ptr(f), ctypes.byref(vc), ctypes.byref(vu))
    return r, vc.value, vu.value


def window_end_area(W, H, x, y, i0, area, k):
    """End (exclusive) of the adaptive window starting at event i0: one past
    the event that brings some area x area square to k events, or len(x)."""
    x = np.ascontiguousarray(x, np.uint16)
    y = np.ascontiguousarray(y, np.uint16)
    return int(_load().oref_window_end_area(int(W), int(H), _ptr(x), _ptr(y), x.size, int(i0), int(area), int(k)))


def alpha_from_dsat(d_sat, eps=1.0 / 255.0):
    """Equation (2): alpha = -d_sat / ln(eps); eq. (3) is eps = 1/255."""
    return -float(d_sat) / float(np.log(eps))


# --------------------------------------------------------------------------
# Pyramid and flow
# --------------------------------------------------------------------------
def level_sizes(W, H, L):
    sizes = []
    for _ in range(L):
        sizes.append((W, H))
        W, H = (W + 1) // 2, (H + 1) // 2
    return sizes


def pyr_down(img):
    img = np.ascontiguousarray(img, np.float32)
    H, W = img.shape
    out = np.empty(((H + 1) // 2, (W + 1) // 2), np.float32)
    _load().oref_pyr_down(W, H, _ptr(img), _ptr(out))
    return out


def pyramid(S, L):
    """Packed pyramid (level 0 first) as one float32 vector, plus the levels."""
    levels = [np.ascontiguousarray(S, np.float32)]
    for _ in range(L - 1):
        levels.append(pyr_down(levels[-1]))
    return np.concatenate([lv.ravel() for lv in levels]), levels


def patch_count(W, H, ps=8, stride=4):
    return int(_load().oref_patch_count(W, H, ps, stride))


class VarParams(ctypes.Structure):
    _fields_ = [("outer", ctypes.c_int32), ("inner", ctypes.c_int32), ("alpha", ctypes.c_double),
                ("gamma", ctypes.c_double), ("delta", ctypes.c_double), ("omega", ctypes.c_double)]


# dense inverse search's usual refinement settings (5 fixed-point iterations
# of 5 SOR sweeps, smoothness 20, gradient constancy 10, brightness 5, 1.6)
VAR_DEFAULT = dict(outer=5, inner=5, alpha=20.0, gamma=10.0, delta=5.0, omega=1.6)


def var_refine(I0, I1, U, outer=5, inner=5, alpha=20.0, gamma=10.0, delta=5.0, omega=1.6):
    """Variational refinement of the dense flow U ([2,H,W], float64; a
    refined copy is returned) between the level images I0 and I1."""
    I0 = np.ascontiguousarray(I0, np.float32)
    I1 = np.ascontiguousarray(I1, np.float32)
    H, W = I0.shape
    out = np.array(U, np.float64, copy=True, order="C")
    assert out.shape == (2, H, W)
    _load().oref_var_refine(W, H, _ptr(I0), _ptr(I1), _ptr(out), int(outer), int(inner), float(alpha),
                            float(gamma), float(delta), float(omega))
    return out


def dis_flow(pyr0, pyr1, W, H, L, ps=8, stride=4, iters=16, lam=0.3,
             want_patches=False, prev_flow=None, refine=None):
    """Dense inverse search flow from pyr0 (window k-1) to pyr1 (window k).
    Returns float64 [2,H,W] (u, v), and per-level patch flows if asked.
    prev_flow: None, or the previous pair's dense [2,H,W] flow, from which
    the coarsest level starts (warm start).  refine: None, or a dict of
    var_refine settings applied to every level's dense flow."""
    pyr0 = np.ascontiguousarray(pyr0, np.float32)
    pyr1 = np.ascontiguousarray(pyr1, np.float32)
    flow = np.empty((2, H, W), np.float64)
    npatch = sum(patch_count(w, h, ps, stride) for w, h in level_sizes(W, H, L))
    pu = np.empty((npatch, 2), np.float64) if want_patches else None
    warm = None
    if prev_flow is not None:
        warm = np.ascontiguousarray(prev_flow, np.float64)
        assert warm.shape == (2, H, W)
    vr = None
    if refine is not None:
        vr = VarParams(**{**VAR_DEFAULT, **refine})
    rc = _load().oref_dis_flow_refined(W, H, L, _ptr(pyr0), _ptr(pyr1), ps, stride,
                                       iters, float(lam), _ptr(warm) if warm is not None else None,
                                       ctypes.byref(vr) if vr is not None else None,
                                       _ptr(flow), _ptr(pu) if pu is not None else None)
    if rc != 0:
        raise ValueError("oref_dis_flow rejected its arguments")
    if want_patches:
        return flow, pu
    return flow


# Update-prediction filter (Sec. III-D's flow block, Sec. IV-A's layer
# parameters): the reading is spelled out in ebof_oracle.h.
def ff_transport(U):
    """The previous flow U ([2,H,W]) carried along itself over one window:
    P(x) = U(x - U(x)), bilinear with replicated border."""
    U = np.ascontiguousarray(U, np.float64)
    _, H, W = U.shape
    P = np.empty_like(U)
    _load().oref_ff_transport(W, H, _ptr(U), _ptr(P))
    return P


def ff_smooth(F, iters):
    """`iters` Jacobi iterations of the five-point mean (replicated border)
    on both planes of F ([2,H,W]); a smoothed copy is returned."""
    out = np.array(F, np.float64, copy=True, order="C")
    _, H, W = out.shape
    _load().oref_ff_smooth(W, H, int(iters), _ptr(out))
    return out


def filter_state_size(W, H, layers):
    """Doubles (and floats on the GPU) of a filter state of `layers` layers."""
    return sum(2 * w * h for w, h in level_sizes(W, H, layers))


def flow_filter(pyr0, pyr1, W, H, L, gamma, smooth, state=None):
    """One step of the update-prediction filter from pyr0 (window k-1) to
    pyr1 (window k), both L-level pyramids.  gamma / smooth: per layer, layer
    0 the finest; their length is the number of layers.  state: the previous
    step's flat state (None: zero).  Returns (flow [2,H,W] float64, state)."""
    pyr0 = np.ascontiguousarray(pyr0, np.float32)
    pyr1 = np.ascontiguousarray(pyr1, np.float32)
    F = len(gamma)
    assert len(smooth) == F
    n = filter_state_size(W, H, F)
    st = np.zeros(n, np.float64) if state is None else np.array(state, np.float64, copy=True, order="C")
    assert st.shape == (n,)
    g = np.ascontiguousarray(gamma, np.float64)
    sm = np.ascontiguousarray(smooth, np.int32)
    flow = np.empty((2, H, W), np.float64)
    rc = _load().oref_flow_filter(W, H, L, _ptr(pyr0), _ptr(pyr1), F, _ptr(g), _ptr(sm), _ptr(st), _ptr(flow))
    if rc != 0:
        raise ValueError("oref_flow_filter rejected its arguments")
    return flow, st


def filter_layer(state, W, H, l):
    """Layer l ([2,H_l,W_l]) of a flat filter state."""
    sizes = level_sizes(W, H, l + 1)
    off = sum(2 * w * h for w, h in sizes[:l])
    w, h = sizes[l]
    return np.asarray(state)[off:off + 2 * w * h].reshape(2, h, w)


def _patch_grid(W, H, ps, stride):
    return (W - ps + stride - 1) // stride + 1, (H - ps + stride - 1) // stride + 1


def patch_init_coarser(W, H, Uc, ps=8, stride=4):
    """Initial patch displacements [ny, nx, 2] of a W x H level from the
    coarser level's dense flow Uc [2, Hc, Wc]."""
    Uc = np.ascontiguousarray(Uc, np.float64)
    nx, ny = _patch_grid(W, H, ps, stride)
    u0 = np.empty((ny, nx, 2), np.float64)
    _load().oref_patch_init_coarser(W, H, ps, stride, _ptr(Uc), Uc.shape[2], Uc.shape[1], _ptr(u0))
    return u0


def patch_init_previous(W, H, level, Up, ps=8, stride=4):
    """Initial patch displacements [ny, nx, 2] of level `level` (W x H) from
    the previous pair's dense level-0 flow Up [2, H0, W0] (warm start)."""
    Up = np.ascontiguousarray(Up, np.float64)
    nx, ny = _patch_grid(W, H, ps, stride)
    u0 = np.empty((ny, nx, 2), np.float64)
    _load().oref_patch_init_previous(W, H, int(level), ps, stride, _ptr(Up), Up.shape[2], Up.shape[1],
                                     _ptr(u0))
    return u0


def dis_level(I0, I1, u0=None, ps=8, stride=4, iters=16, lam=0.3):
    """Patch inverse search on one level (images [H, W] float32) from the
    initial displacements u0 [ny, nx, 2] (None = 0); returns [ny, nx, 2]."""
    I0 = np.ascontiguousarray(I0, np.float32)
    I1 = np.ascontiguousarray(I1, np.float32)
    H, W = I0.shape
    nx, ny = _patch_grid(W, H, ps, stride)
    pu = np.empty((ny, nx, 2), np.float64)
    if u0 is not None:
        u0 = np.ascontiguousarray(u0, np.float64)
        assert u0.shape == (ny, nx, 2)
    _load().oref_dis_level(W, H, _ptr(I0), _ptr(I1), ps, stride, int(iters), float(lam),
                           _ptr(u0) if u0 is not None else None, _ptr(pu))
    return pu


def densify(I0, I1, pu, ps=8, stride=4):
    """Dense flow [2, H, W] from patch displacements pu [ny, nx, 2]."""
    I0 = np.ascontiguousarray(I0, np.float32)
    I1 = np.ascontiguousarray(I1, np.float32)
    H, W = I0.shape
    nx, ny = _patch_grid(W, H, ps, stride)
    pu = np.ascontiguousarray(pu, np.float64)
    assert pu.shape == (ny, nx, 2)
    U = np.empty((2, H, W), np.float64)
    _load().oref_densify(W, H, _ptr(I0), _ptr(I1), ps, stride, _ptr(pu), _ptr(U))
    return U


# --------------------------------------------------------------------------
# The whole per-window path (events -> E_df -> D2 -> S -> pyramid)
# --------------------------------------------------------------------------
def window(W, H, x, y, t, t0, dt, n_d, n_f, alpha, L):
    """Returns dict(E=raw edge image, Edf, D2, S, pyr (packed), dropped)."""
    E, dropped = edge_image(W, H, x, y, t, t0, dt)
    Edf = denoise_fill(E, n_d, n_f)
    D2 = edt_separable(Edf)
    S = surface(D2, alpha)
    pyr, _ = pyramid(S, L)
    return dict(E=E, Edf=Edf, D2=D2, S=S, pyr=pyr, dropped=dropped)
