"""Thin Python binding: one function per C entry point, same names.

Each function only checks tensor placement/dtype, marshals pointers and the
current HIP stream, calls the library and raises on a non-OK status.  Every
computation happens in the library's kernels; PyTorch supplies device memory
and the stream.
"""

from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import PgsCamera, PgsReplay, PgsViewBatch, check


def _ptr(t, dtype=None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor):
        raise TypeError("expected a torch tensor")
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"expected {dtype}, got {t.dtype}")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def camera_struct(cam: dict) -> PgsCamera:
    c = PgsCamera()
    c.width = int(cam["width"])
    c.height = int(cam["height"])
    c.fx, c.fy, c.cx, c.cy = (float(cam[k]) for k in ("fx", "fy", "cx", "cy"))
    vm = np.asarray(cam["viewmat"], np.float32).reshape(12)
    for i in range(12):
        c.viewmat[i] = float(vm[i])
    return c


def replay_struct(trace) -> PgsReplay | None:
    if trace is None:
        return None
    r = PgsReplay()
    r.mask_dev = _ptr(trace["mask"], torch.int64).value
    r.steps_dev = _ptr(trace["steps"], torch.int32).value
    r.base_dev = _ptr(trace["base"], torch.int32).value
    r.used_dev = _ptr(trace["used"], torch.int64).value
    r.entry_dev = _ptr(trace["entry"], torch.float32).value
    _need(trace["steps"], trace["base"].numel(), "trace base")
    words = int(trace["entry"].shape[1])
    _need(trace["entry"], words * int(trace["entry_capacity"]), "trace entries")
    _need(trace["mask"], int(trace["pair_capacity"]) * trace["steps"].shape[-1], "trace masks")
    r.count_dev = _ptr(trace["count"], torch.int32).value
    r.entry_capacity = int(trace["entry_capacity"])
    r.pair_capacity = int(trace["pair_capacity"])
    r.entry_words = words
    return r


def pgs_trace_entries(pair_capacity, tile_w, tile_h) -> int:
    return int(_lib.load().pgs_trace_entries(pair_capacity, tile_w, tile_h))


def _f3(v):
    return (ctypes.c_float * 3)(*[float(x) for x in v])


F32, I32, I64 = torch.float32, torch.int32, torch.int64


def pgs_version() -> str:
    return _lib.load().pgs_version().decode()


def pgs_check_flags(flags, stream=None) -> tuple[int, int]:
    """Waits for the stream and reads the device flags word: (status, word),
    status PGS_OK or PGS_ERR_CAPACITY (a pair or trace buffer overflowed);
    raises on any other status."""
    host = ctypes.c_uint32(0)
    st = _lib.load().pgs_check_flags(_ptr(flags, I32), ctypes.byref(host), _stream(stream))
    if st not in (_lib.PGS_OK, _lib.PGS_ERR_CAPACITY):
        check(st, "pgs_check_flags")
    return int(st), int(host.value)


def pgs_graph_begin(stream):
    check(_lib.load().pgs_graph_begin(_stream(stream)), "pgs_graph_begin")


def pgs_graph_end(stream) -> ctypes.c_void_p:
    """Ends the capture begun on `stream`; returns the instantiated graph's
    handle (free it with pgs_graph_destroy)."""
    h = ctypes.c_void_p()
    check(_lib.load().pgs_graph_end(_stream(stream), ctypes.byref(h)), "pgs_graph_end")
    return h


def pgs_graph_launch(graph, stream=None):
    check(_lib.load().pgs_graph_launch(graph, _stream(stream)), "pgs_graph_launch")


def pgs_graph_destroy(graph):
    if graph is not None and graph.value:
        _lib.load().pgs_graph_destroy(graph)


def pgs_project(params, n, sh_degree, cam, tile_w, tile_h, proj, radius, rect, touched, stream=None):
    lib = _lib.load()
    c = camera_struct(cam)
    _need(params, (11 + 3 * (sh_degree + 1) ** 2) * n, "params")
    _need(proj, 16 * n, "proj")
    _need(radius, n, "radius")
    _need(rect, 2 * n, "rect")
    _need(touched, n, "touched")
    check(lib.pgs_project(_ptr(params, F32), n, sh_degree, ctypes.byref(c), tile_w, tile_h,
                          _ptr(proj, F32), _ptr(radius, I32), _ptr(rect, I32), _ptr(touched, I32),
                          _stream(stream)), "pgs_project")


def pgs_bin_sort_workspace(n, capacity) -> int:
    return int(_lib.load().pgs_bin_sort_workspace(n, capacity))


def pgs_bin_sort(n, proj, rect, touched, tiles_x, n_tiles, view_tile_offset, capacity, keys, values,
                 ranges, num_pairs, flags, workspace, stream=None):
    lib = _lib.load()
    _need(proj, 16 * n, "proj")
    _need(ranges, 2 * n_tiles, "ranges")
    check(lib.pgs_bin_sort(n, _ptr(proj, F32), _ptr(rect, I32), _ptr(touched, I32), tiles_x, n_tiles,
                           view_tile_offset, capacity, _ptr(keys, I64), _ptr(values, I32),
                           _ptr(ranges, I32), _ptr(num_pairs, I32), _ptr(flags, I32),
                           _ptr(workspace, torch.uint8), workspace.numel(), _stream(stream)),
          "pgs_bin_sort")


def pgs_sort_workspace(capacity) -> int:
    return int(_lib.load().pgs_sort_workspace(capacity))


def pgs_sort_pairs(keys, values, count, capacity, key_bits, workspace, stream=None):
    lib = _lib.load()
    check(lib.pgs_sort_pairs(_ptr(keys, I64), _ptr(values, I32), _ptr(count, I32), capacity, key_bits,
                             _ptr(workspace, torch.uint8), workspace.numel(), _stream(stream)),
          "pgs_sort_pairs")


def pgs_sort_pairs_noalloc(keys, values, count, capacity, key_bits, stream=None):
    lib = _lib.load()
    check(lib.pgs_sort_pairs_noalloc(_ptr(keys, I64), _ptr(values, I32), _ptr(count, I32), capacity, key_bits,
                                     _stream(stream)), "pgs_sort_pairs_noalloc")


def pgs_tile_order(ranges, tiles_in_view, view_tile_offset, n_tiles, order, stream=None):
    lib = _lib.load()
    check(lib.pgs_tile_order(_ptr(ranges, I32), tiles_in_view, view_tile_offset, n_tiles,
                             _ptr(order, I32), _stream(stream)), "pgs_tile_order")


def pgs_render_fwd(width, height, tile_w, tile_h, proj, n, values, ranges, view_tile_offset, bg,
                   image, t_final, n_contrib, trace, flags, tile_order=None, stream=None):
    lib = _lib.load()
    _need(proj, 16 * n, "proj")
    _need(image, 3 * width * height, "image")
    _need(t_final, width * height, "t_final")
    _need(n_contrib, width * height, "n_contrib")
    r = replay_struct(trace)
    check(lib.pgs_render_fwd(width, height, tile_w, tile_h, _ptr(proj, F32), n, _ptr(values, I32),
                             _ptr(ranges, I32), view_tile_offset, _f3(bg), _ptr(image, F32),
                             _ptr(t_final, F32), _ptr(n_contrib, I32),
                             ctypes.byref(r) if r is not None else None, _ptr(flags, I32),
                             _ptr(tile_order, I32), _stream(stream)), "pgs_render_fwd")


def pgs_render_bwd(width, height, tile_w, tile_h, proj, n, values, ranges, view_tile_offset, bg,
                   t_final, n_contrib, trace, dl_dimage, grad2d, tile_order=None, stream=None):
    lib = _lib.load()
    _need(proj, 16 * n, "proj")
    _need(grad2d, 16 * n, "grad2d")
    _need(dl_dimage, 3 * width * height, "dl_dimage")
    r = replay_struct(trace)
    check(lib.pgs_render_bwd(width, height, tile_w, tile_h, _ptr(proj, F32), n, _ptr(values, I32),
                             _ptr(ranges, I32), view_tile_offset, _f3(bg), _ptr(t_final, F32),
                             _ptr(n_contrib, I32), ctypes.byref(r) if r is not None else None,
                             _ptr(dl_dimage, F32), _ptr(grad2d, F32), _ptr(tile_order, I32),
                             _stream(stream)), "pgs_render_bwd")


def pgs_project_bwd(params, n, sh_degree, cam, radius, grad2d, grads, stream=None):
    lib = _lib.load()
    c = camera_struct(cam)
    _need(grad2d, 16 * n, "grad2d")
    _need(grads, (11 + 3 * (sh_degree + 1) ** 2) * n, "grads")
    check(lib.pgs_project_bwd(_ptr(params, F32), n, sh_degree, ctypes.byref(c), _ptr(radius, I32),
                              _ptr(grad2d, F32), _ptr(grads, F32), _stream(stream)), "pgs_project_bwd")


def pgs_loss_workspace(width, height) -> int:
    return int(_lib.load().pgs_loss_workspace(width, height))


def pgs_loss_l1_dssim(x, y, width, height, lam, loss, dl_dx, workspace, stream=None):
    lib = _lib.load()
    check(lib.pgs_loss_l1_dssim(_ptr(x, F32), _ptr(y, F32), width, height, float(lam), _ptr(loss, F32),
                                _ptr(dl_dx, F32), _ptr(workspace, torch.uint8), workspace.numel(),
                                _stream(stream)), "pgs_loss_l1_dssim")


def pgs_psnr(x, y, width, height, out, workspace, stream=None):
    lib = _lib.load()
    check(lib.pgs_psnr(_ptr(x, F32), _ptr(y, F32), width, height, _ptr(out, F32),
                       _ptr(workspace, torch.uint8), workspace.numel(), _stream(stream)), "pgs_psnr")


def pgs_adam_step(params, grads, m, v, rows, n, lr, step, beta1, beta2, eps, stream=None):
    lib = _lib.load()
    lr_arr = (ctypes.c_float * rows)(*[float(x) for x in lr])
    check(lib.pgs_adam_step(_ptr(params, F32), _ptr(grads, F32), _ptr(m, F32), _ptr(v, F32), rows, n,
                            lr_arr, int(step), float(beta1), float(beta2), float(eps), _stream(stream)),
          "pgs_adam_step")


def pgs_knn_workspace(m) -> int:
    return int(_lib.load().pgs_knn_workspace(m))


def pgs_knn(points, m, k, nbr, d2, workspace, stream=None):
    lib = _lib.load()
    check(lib.pgs_knn(_ptr(points, F32), m, k, _ptr(nbr, I32), _ptr(d2, torch.float64),
                      _ptr(workspace, torch.uint8), workspace.numel(), _stream(stream)), "pgs_knn")


def pgs_atomic_scatter(records, n_records, targets, n_targets, stream=None):
    _need(records, 16 * n_records, "records")
    _need(targets, n_targets, "targets")
    check(_lib.load().pgs_atomic_scatter(_ptr(records, F32), n_records, _ptr(targets, I32), n_targets,
                                         _stream(stream)), "pgs_atomic_scatter")


def pgs_stream_copy(src, dst, nbytes, stream=None):
    lib = _lib.load()
    check(lib.pgs_stream_copy(_ptr(src), _ptr(dst), int(nbytes), _stream(stream)), "pgs_stream_copy")


def pgs_pca_seed(points, colours, m, nbr, d2, k, r_normal, params, stream=None):
    lib = _lib.load()
    check(lib.pgs_pca_seed(_ptr(points, F32), _ptr(colours, F32), m, _ptr(nbr, I32),
                           _ptr(d2, torch.float64), k, float(r_normal), _ptr(params, F32),
                           _stream(stream)), "pgs_pca_seed")


def _need(t, count, what):
    if t is not None and t.numel() < count:
        raise ValueError(f"{what}: {t.numel()} elements, need {count}")


N_MLP_WEIGHTS = 13000


def pgs_mlp_weight_count():
    return int(_lib.load().pgs_mlp_weight_count())


def pgs_mlp_features(points, m, nbr, d2, k, r_normal, x, base, stream=None):
    lib = _lib.load()
    _need(points, 3 * m, "points")
    _need(nbr, k * m, "nbr")
    _need(d2, k * m, "d2")
    _need(x, 64 * m, "x")
    _need(base, 16 * m, "base")
    check(lib.pgs_mlp_features(_ptr(points, F32), m, _ptr(nbr, I32), _ptr(d2, torch.float64), k,
                               float(r_normal), _ptr(x, F32), _ptr(base, F32), _stream(stream)),
          "pgs_mlp_features")


def pgs_mlp_forward(weights, x, m, y, stream=None):
    lib = _lib.load()
    _need(weights, N_MLP_WEIGHTS, "weights")
    _need(x, 64 * m, "x")
    _need(y, 8 * m, "y")
    check(lib.pgs_mlp_forward(_ptr(weights, F32), _ptr(x, F32), m, _ptr(y, F32), _stream(stream)),
          "pgs_mlp_forward")


def pgs_mlp_backward_workspace(m):
    return int(_lib.load().pgs_mlp_backward_workspace(m))


def pgs_mlp_backward(weights, x, m, dy, dweights, workspace, stream=None):
    lib = _lib.load()
    _need(weights, N_MLP_WEIGHTS, "weights")
    _need(dweights, N_MLP_WEIGHTS, "dweights")
    _need(x, 64 * m, "x")
    _need(dy, 8 * m, "dy")
    check(lib.pgs_mlp_backward(_ptr(weights, F32), _ptr(x, F32), m, _ptr(dy, F32), _ptr(dweights, F32),
                               _ptr(workspace, torch.uint8), workspace.numel(), _stream(stream)),
          "pgs_mlp_backward")


def pgs_seed_targets(params, n, targets, stream=None):
    lib = _lib.load()
    _need(params, 11 * n, "params")
    _need(targets, 8 * n, "targets")
    check(lib.pgs_seed_targets(_ptr(params, F32), n, _ptr(targets, F32), _stream(stream)), "pgs_seed_targets")


def pgs_seed_loss_workspace(m):
    return int(_lib.load().pgs_seed_loss_workspace(m))


def pgs_seed_loss(y, base, target, m, scale, loss, dy, workspace, stream=None):
    lib = _lib.load()
    _need(y, 8 * m, "y")
    _need(base, 16 * m, "base")
    _need(target, 8 * m, "target")
    _need(dy, 8 * m, "dy")
    _need(loss, 1, "loss")
    check(lib.pgs_seed_loss(_ptr(y, F32), _ptr(base, F32), _ptr(target, F32), m, float(scale),
                            _ptr(loss, F32), _ptr(dy, F32), _ptr(workspace, torch.uint8), workspace.numel(),
                            _stream(stream)), "pgs_seed_loss")


def pgs_seed_apply(y, base, pca_params, m, params, fallback=None, fallback_count=None, stream=None):
    lib = _lib.load()
    _need(y, 8 * m, "y")
    _need(base, 16 * m, "base")
    _need(pca_params, 14 * m, "pca_params")
    _need(params, 14 * m, "params")
    _need(fallback, m, "fallback")
    _need(fallback_count, 1, "fallback_count")
    check(lib.pgs_seed_apply(_ptr(y, F32), _ptr(base, F32), _ptr(pca_params, F32), m, _ptr(params, F32),
                             _ptr(fallback, torch.uint8), _ptr(fallback_count, I32), _stream(stream)),
          "pgs_seed_apply")


class ViewBatch:
    """A pgs_view_batch and the camera array it points to (kept alive here),
    with the batch layout: tile_offsets / pixel_offsets [n_views + 1]."""

    def __init__(self, cams, tile=(16, 16), batch=256, blocks=0):
        self.cams = list(cams)
        self.tile_w, self.tile_h = int(tile[0]), int(tile[1])
        self.batch, self.blocks = int(batch), int(blocks)
        v = len(self.cams)
        self._arr = (PgsCamera * v)(*[camera_struct(c) for c in self.cams])
        self.struct = PgsViewBatch(v, ctypes.cast(self._arr, ctypes.POINTER(PgsCamera)), self.tile_w,
                                   self.tile_h, self.batch, self.blocks)
        to = (ctypes.c_int32 * (v + 1))()
        po = (ctypes.c_int64 * (v + 1))()
        total = _lib.load().pgs_views_layout(ctypes.byref(self.struct), to, po)
        if total < 0:
            raise ValueError(_lib.load().pgs_last_error().decode())
        self.tile_offsets = list(to)
        self.pixel_offsets = list(po)
        self.n_tiles = int(total)
        self.n_pixels = int(po[v])

    @property
    def n_views(self):
        return len(self.cams)


def pgs_project_views(views, params, n, sh_degree, proj_all, radius_all, rect_all, touched_all, stream=None):
    lib = _lib.load()
    V = views.n_views
    _need(params, (11 + 3 * (sh_degree + 1) ** 2) * n, "params")
    _need(proj_all, V * 16 * n, "proj_all")
    _need(radius_all, V * n, "radius_all")
    _need(rect_all, V * 2 * n, "rect_all")
    _need(touched_all, V * n, "touched_all")
    check(lib.pgs_project_views(ctypes.byref(views.struct), _ptr(params, F32), n, sh_degree, _ptr(proj_all, F32),
                                _ptr(radius_all, I32), _ptr(rect_all, I32), _ptr(touched_all, I32),
                                _stream(stream)), "pgs_project_views")


def pgs_project_bwd_views(views, params, n, sh_degree, radius_all, grad2d_all, grads, stream=None):
    lib = _lib.load()
    V = views.n_views
    _need(params, (11 + 3 * (sh_degree + 1) ** 2) * n, "params")
    _need(radius_all, V * n, "radius_all")
    _need(grad2d_all, V * 16 * n, "grad2d_all")
    _need(grads, (11 + 3 * (sh_degree + 1) ** 2) * n, "grads")
    check(lib.pgs_project_bwd_views(ctypes.byref(views.struct), _ptr(params, F32), n, sh_degree,
                                    _ptr(radius_all, I32), _ptr(grad2d_all, F32), _ptr(grads, F32),
                                    _stream(stream)), "pgs_project_bwd_views")


def pgs_bin_sort_views(views, n, proj_all, rect_all, touched_all, capacity, keys, values, ranges, num_pairs,
                       flags, workspace, stream=None):
    lib = _lib.load()
    _need(ranges, 2 * views.n_tiles, "ranges")
    _need(proj_all, views.n_views * 16 * n, "proj_all")
    _need(keys, capacity, "keys")
    _need(values, capacity, "values")
    check(lib.pgs_bin_sort_views(ctypes.byref(views.struct), n, _ptr(proj_all, F32), _ptr(rect_all, I32),
                                 _ptr(touched_all, I32), int(capacity), _ptr(keys, I64), _ptr(values, I32),
                                 _ptr(ranges, I32), _ptr(num_pairs, I32), _ptr(flags, I32),
                                 _ptr(workspace, torch.uint8), workspace.numel(), _stream(stream)),
          "pgs_bin_sort_views")


def pgs_render_fwd_views(views, proj_all, n, values, ranges, bg, image_all, t_final_all, n_contrib_all, trace,
                         flags, tile_order, queue, stream=None):
    lib = _lib.load()
    _need(image_all, 3 * views.n_pixels, "image_all")
    _need(t_final_all, views.n_pixels, "t_final_all")
    _need(n_contrib_all, views.n_pixels, "n_contrib_all")
    _need(tile_order, views.n_tiles, "tile_order")
    bg_arr = (ctypes.c_float * 3)(*[float(x) for x in bg])
    rep = replay_struct(trace)
    check(lib.pgs_render_fwd_views(ctypes.byref(views.struct), _ptr(proj_all, F32), n, _ptr(values, I32),
                                   _ptr(ranges, I32), bg_arr, _ptr(image_all, F32), _ptr(t_final_all, F32),
                                   _ptr(n_contrib_all, I32), ctypes.byref(rep) if rep is not None else None,
                                   _ptr(flags, I32), _ptr(tile_order, I32), _ptr(queue, I32), _stream(stream)),
          "pgs_render_fwd_views")


def pgs_render_bwd_views(views, proj_all, n, values, ranges, bg, t_final_all, n_contrib_all, trace, dl_all,
                         grad2d_all, tile_order, queue, stream=None):
    lib = _lib.load()
    _need(dl_all, 3 * views.n_pixels, "dl_all")
    _need(grad2d_all, views.n_views * 16 * n, "grad2d_all")
    _need(tile_order, views.n_tiles, "tile_order")
    bg_arr = (ctypes.c_float * 3)(*[float(x) for x in bg])
    rep = replay_struct(trace)
    check(lib.pgs_render_bwd_views(ctypes.byref(views.struct), _ptr(proj_all, F32), n, _ptr(values, I32),
                                   _ptr(ranges, I32), bg_arr, _ptr(t_final_all, F32), _ptr(n_contrib_all, I32),
                                   ctypes.byref(rep) if rep is not None else None, _ptr(dl_all, F32),
                                   _ptr(grad2d_all, F32), _ptr(tile_order, I32), _ptr(queue, I32),
                                   _stream(stream)),
          "pgs_render_bwd_views")


def pgs_adam_step_dev(params, grads, m, v, rows, n, lr, state, beta1, beta2, eps, stream=None):
    lib = _lib.load()
    _need(state, 4, "state")
    lr_arr = (ctypes.c_float * rows)(*[float(x) for x in lr])
    check(lib.pgs_adam_step_dev(_ptr(params, F32), _ptr(grads, F32), _ptr(m, F32), _ptr(v, F32), rows, n,
                                lr_arr, _ptr(state, I32), float(beta1), float(beta2), float(eps),
                                _stream(stream)), "pgs_adam_step_dev")
