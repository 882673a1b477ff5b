"""Python front end of the MI355X surfel feature rasterizer.

PyTorch supplies device memory and the current HIP stream; every stage runs
in the HIP library through the C ABI (see include/fastsegsim.h):

    preprocess -> bin -> sort -> render_forward  (-> render_backward)

The Rasterizer owns the per-frame buffers (records, key/value pairs, tile
ranges, workspace) and grows the pair buffers when a frame needs more.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import torch

from . import _lib as L

ALPHA_MIN = 1.0 / 255.0
ALPHA_MAX = 0.99
T_STOP = 1e-4


def _p(t: torch.Tensor | None):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(device) -> ctypes.c_void_p:
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


def _f32(t: torch.Tensor, shape, name: str) -> torch.Tensor:
    if t.dtype != torch.float32 or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must be a contiguous float32 tensor of shape {tuple(shape)}, got "
                         f"{t.dtype} {tuple(t.shape)}")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on the GPU")
    return t


@dataclass
class Frame:
    """Outputs (and intermediates) of one rendered frame."""
    feat: torch.Tensor          # (total_pixels, C) float32
    T: torch.Tensor             # (total_pixels,) float32
    n: torch.Tensor             # (total_pixels,) int32
    last: torch.Tensor | None   # (total_pixels,) int32
    idx: torch.Tensor | None    # (total_pixels, K) int32
    num_pairs: int
    records: torch.Tensor
    tiles_touched: torch.Tensor
    keys: torch.Tensor          # sorted, first num_pairs valid
    vals: torch.Tensor
    ranges: torch.Tensor        # (total_tiles, 2)
    generation: int = -1        # which fill of the rasterizer's shared buffers the frame read
    depth: torch.Tensor | None = None    # (total_pixels,) sum of w z (intersection depths)
    normal: torch.Tensor | None = None   # (total_pixels, 3) sum of w n (camera-space normals)

    def view_image(self, rast: "Rasterizer", v: int = 0, what: str = "feat") -> torch.Tensor:
        cam = rast.cam_arr[v]
        a = getattr(self, what)
        sl = a[cam.pixel_offset: cam.pixel_offset + cam.width * cam.height]
        return sl.reshape((cam.height, cam.width) + tuple(a.shape[1:]))


class Rasterizer:
    """Renders C-channel feature images of a surfel scene from one or more views."""

    def __init__(self, cams, *, tile: int = 16, topk: int = 0, tile_mode: str = "precise",
                 feat_dtype: str = "f32", alpha_min: float = ALPHA_MIN, alpha_max: float = ALPHA_MAX,
                 t_stop: float = T_STOP, batch: int = 0, schedule: str = "auto", topk_mode: str = "first",
                 lowpass: bool = False, device: str | torch.device = "cuda", pair_capacity: int = 0):
        self.lib = L.load()
        self.device = torch.device(device)
        self.cams = list(cams) if isinstance(cams, (list, tuple)) else [cams]
        self.num_views = len(self.cams)
        mode = {"precise": L.FS_TILES_PRECISE, "bbox": L.FS_TILES_BBOX, "linearised": L.FS_TILES_LINEARISED}[tile_mode]
        dt = {"f32": L.FS_FEAT_F32, "bf16": L.FS_FEAT_BF16}[feat_dtype]
        self.feat_dtype = feat_dtype
        if schedule == "auto":   # the measured fastest: split for Top-K, the longest-first queue for the full blend
            schedule = "split" if topk > 0 else "persistent"
        sched = {"grid": L.FS_SCHED_GRID, "persistent": L.FS_SCHED_PERSISTENT, "split": L.FS_SCHED_SPLIT}[schedule]
        kmode = {"first": L.FS_TOPK_FIRST, "weight": L.FS_TOPK_WEIGHT}[topk_mode]
        self.opts = L.make_opts(tile, topk, mode, dt, alpha_min, alpha_max, t_stop, batch, sched, kmode, int(lowpass))
        self.cam_arr, self.total_tiles, self.total_pixels = L.make_cameras(self.cams, tile)
        raw = bytes(ctypes.string_at(ctypes.addressof(self.cam_arr), ctypes.sizeof(self.cam_arr)))
        self.cams_dev = torch.frombuffer(bytearray(raw), dtype=torch.uint8).to(self.device)
        self.capacity = int(pair_capacity)
        self._n = -1
        self._bufs: dict[str, torch.Tensor] = {}
        # records, pairs and ranges are shared by every frame this object
        # renders; each preprocess refills them and bumps the generation, so a
        # backward can tell whether its frame's lists are still the ones held
        self.generation = 0

    @property
    def topk(self) -> int:
        return int(self.opts.topk)

    def set_cameras(self, cams) -> None:
        """Replace the camera poses/intrinsics in place (same resolutions), so a
        captured frame graph renders the new views on its next replay."""
        cams = list(cams) if isinstance(cams, (list, tuple)) else [cams]
        if [(c.width, c.height) for c in cams] != [(c.width, c.height) for c in self.cams]:
            raise ValueError("set_cameras keeps the view resolutions")
        arr, tt, tp = L.make_cameras(cams, int(self.opts.tile))
        raw = bytes(ctypes.string_at(ctypes.addressof(arr), ctypes.sizeof(arr)))
        self.cams_dev.copy_(torch.frombuffer(bytearray(raw), dtype=torch.uint8))
        self.cams, self.cam_arr = cams, arr

    # -- buffers ------------------------------------------------------------
    def _ensure(self, n: int, capacity: int):
        if n != self._n:
            V = self.num_views
            self._bufs["records"] = torch.empty(V * n * L.FS_RECORD_BYTES, dtype=torch.uint8, device=self.device)
            self._bufs["tiles"] = torch.empty(V * n, dtype=torch.int32, device=self.device)
            self._bufs["tile_cache"] = torch.empty(V * n * L.FS_TILE_CACHE_WORDS, dtype=torch.int32,
                                                   device=self.device)
            self._bufs["num_pairs"] = torch.zeros(1, dtype=torch.int64, device=self.device)
            self._bufs["ranges"] = torch.empty(self.total_tiles * 2, dtype=torch.int32, device=self.device)
            self._n = n
        if capacity > self.capacity or "keys" not in self._bufs:
            self.capacity = max(capacity, self.capacity, 1024)
            self._bufs["keys"] = torch.empty(self.capacity, dtype=torch.int64, device=self.device)
            self._bufs["vals"] = torch.empty(self.capacity, dtype=torch.int32, device=self.device)
        ws = self.lib.fs_workspace_bytes(n, self.num_views, self.total_tiles, self.capacity, ctypes.byref(self.opts))
        if "ws" not in self._bufs or self._bufs["ws"].numel() < ws:
            self._bufs["ws"] = torch.empty(max(ws, 256), dtype=torch.uint8, device=self.device)

    # -- stages -------------------------------------------------------------
    def preprocess(self, means, scales, quats, opacity):
        n = means.shape[0]
        self._ensure(n, self.capacity or max(4096, 2 * n * self.num_views))
        b = self._bufs
        self.generation += 1
        L.check(self.lib.fs_preprocess(_p(means), _p(scales), _p(quats), _p(opacity), n, _p(self.cams_dev),
                                       self.num_views, ctypes.byref(self.opts), _p(b["records"]), _p(b["tiles"]),
                                       _p(b["tile_cache"]), _stream(self.device)), "fs_preprocess")
        return b["records"], b["tiles"]

    def bin(self, means, scales, quats, opacity) -> int:
        n = means.shape[0]
        for _ in range(4):
            b = self._bufs
            P = ctypes.c_int64(0)
            st = self.lib.fs_bin(_p(means), _p(scales), _p(quats), _p(opacity), n, _p(self.cams_dev), self.num_views,
                                 ctypes.byref(self.opts), _p(b["tiles"]), _p(b["tile_cache"]), _p(b["keys"]),
                                 _p(b["vals"]), self.capacity, _p(b["num_pairs"]), ctypes.byref(P), _p(b["ws"]),
                                 _stream(self.device))
            if st == L.FS_ERR_CAPACITY:
                self._ensure(n, int(P.value * 1.25) + 1024)
                continue
            L.check(st, "fs_bin")
            return int(P.value)
        raise L.FastSegSimError(L.FS_ERR_CAPACITY, "fs_bin")

    def sort(self, num_pairs: int):
        b = self._bufs
        L.check(self.lib.fs_sort(_p(b["keys"]), _p(b["vals"]), self.capacity, _p(b["num_pairs"]), num_pairs,
                                 self.total_tiles, _p(b["ranges"]), _p(b["ws"]), _stream(self.device)), "fs_sort")
        return b["ranges"]

    def render_forward(self, feats, *, out=None, want_last: bool = False, want_idx: bool = False,
                       want_depth: bool = False, want_normal: bool = False, counters: torch.Tensor | None = None):
        n, C = feats.shape
        if feats.dtype != (torch.bfloat16 if self.feat_dtype == "bf16" else torch.float32) or not feats.is_contiguous():
            raise ValueError(f"feats must be contiguous {self.feat_dtype}")
        b = self._bufs
        dev = self.device
        if out is None:
            out = self.alloc_out(C, want_last=want_last, want_idx=want_idx, want_depth=want_depth,
                                 want_normal=want_normal)
        depth, normal = out.get("depth"), out.get("normal")
        L.check(self.lib.fs_render_forward(_p(b["records"]), _p(b["keys"]) if depth is not None else None,
                                           _p(b["vals"]), _p(b["ranges"]), _p(feats), C, n, _p(self.cams_dev),
                                           self.num_views, self.total_tiles, ctypes.byref(self.opts), _p(out["feat"]),
                                           _p(out["T"]), _p(out["n"]), _p(out["last"]), _p(out["idx"]), _p(depth),
                                           _p(normal), _p(counters), _p(b["ws"]), _stream(dev)),
                "fs_render_forward")
        return out

    def render_labels(self, feats, *, out=None, want_score: bool = True, counters: torch.Tensor | None = None):
        """Per-pixel argmax channel (and its value) of the Top-K render, from
        the current sorted lists; needs the split schedule."""
        n, C = feats.shape
        if feats.dtype != (torch.bfloat16 if self.feat_dtype == "bf16" else torch.float32) or not feats.is_contiguous():
            raise ValueError(f"feats must be contiguous {self.feat_dtype}")
        b = self._bufs
        dev = self.device
        if out is None:
            out = {
                "label": torch.empty(self.total_pixels, dtype=torch.int32, device=dev),
                "score": torch.empty(self.total_pixels, dtype=torch.float32, device=dev) if want_score else None,
                "T": torch.empty(self.total_pixels, dtype=torch.float32, device=dev),
                "n": torch.empty(self.total_pixels, dtype=torch.int32, device=dev),
            }
        L.check(self.lib.fs_render_labels(_p(b["records"]), _p(b["vals"]), _p(b["ranges"]), _p(feats), C, n,
                                          _p(self.cams_dev), self.num_views, self.total_tiles,
                                          ctypes.byref(self.opts), _p(out["label"]), _p(out["score"]), _p(out["T"]),
                                          _p(out["n"]), _p(counters), _p(b["ws"]), _stream(dev)),
                "fs_render_labels")
        return out

    def render(self, means, scales, quats, opacity, feats, *, want_last: bool = False,
               want_idx: bool = False, want_depth: bool = False, want_normal: bool = False) -> Frame:
        n = means.shape[0]
        _f32(means, (n, 3), "means")
        _f32(scales, (n, 2), "scales")
        _f32(quats, (n, 4), "quats")
        _f32(opacity, (n,), "opacity")
        self.preprocess(means, scales, quats, opacity)
        P = self.bin(means, scales, quats, opacity)
        self.sort(P)
        out = self.render_forward(feats, want_last=want_last, want_idx=want_idx, want_depth=want_depth,
                                  want_normal=want_normal)
        b = self._bufs
        return Frame(out["feat"], out["T"], out["n"], out["last"], out["idx"], P, b["records"], b["tiles"],
                     b["keys"], b["vals"], b["ranges"].view(self.total_tiles, 2), self.generation, out.get("depth"),
                     out.get("normal"))

    def render_nosync(self, means, scales, quats, opacity, feats, out: dict, counters=None, events=None) -> None:
        """All four stages without any host synchronisation (the pair count
        stays on the device; launches are sized by the pair capacity, which a
        previous ``render`` call established).  Check ``pairs_fit()`` after."""
        n = means.shape[0]
        b = self._bufs
        if n != self._n or "keys" not in b:
            raise RuntimeError("render_nosync needs a prior render() with the same scene size")
        dev = self.device
        ev = events if events is not None else [None] * 5
        if ev[0] is not None:
            ev[0].record()
        self.generation += 1
        L.check(self.lib.fs_preprocess(_p(means), _p(scales), _p(quats), _p(opacity), n, _p(self.cams_dev),
                                       self.num_views, ctypes.byref(self.opts), _p(b["records"]), _p(b["tiles"]),
                                       _p(b["tile_cache"]), _stream(dev)), "fs_preprocess")
        if ev[1] is not None:
            ev[1].record()
        L.check(self.lib.fs_bin(_p(means), _p(scales), _p(quats), _p(opacity), n, _p(self.cams_dev), self.num_views,
                                ctypes.byref(self.opts), _p(b["tiles"]), _p(b["tile_cache"]), _p(b["keys"]),
                                _p(b["vals"]), self.capacity, _p(b["num_pairs"]), None, _p(b["ws"]), _stream(dev)),
                "fs_bin")
        if ev[2] is not None:
            ev[2].record()
        L.check(self.lib.fs_sort(_p(b["keys"]), _p(b["vals"]), self.capacity, _p(b["num_pairs"]), -1,
                                 self.total_tiles, _p(b["ranges"]), _p(b["ws"]), _stream(dev)), "fs_sort")
        if ev[3] is not None:
            ev[3].record()
        if "label" in out:   # an alloc_labels() dict: the label epilogue in place of the feature image
            self.render_labels(feats, out=out, counters=counters)
        else:
            self.render_forward(feats, out=out, counters=counters)
        if ev[4] is not None:
            ev[4].record()

    def pairs_fit(self) -> bool:
        return int(self._bufs["num_pairs"].item()) <= self.capacity

    def alloc_out(self, C: int, want_last: bool = False, want_idx: bool = False, want_depth: bool = False,
                  want_normal: bool = False) -> dict:
        dev = self.device
        return {
            "feat": torch.empty((self.total_pixels, C), dtype=torch.float32, device=dev),
            "T": torch.empty(self.total_pixels, dtype=torch.float32, device=dev),
            "n": torch.empty(self.total_pixels, dtype=torch.int32, device=dev),
            "last": torch.empty(self.total_pixels, dtype=torch.int32, device=dev) if want_last else None,
            "idx": (torch.empty((self.total_pixels, self.topk), dtype=torch.int32, device=dev)
                    if want_idx and self.topk > 0 else None),
            "depth": torch.empty(self.total_pixels, dtype=torch.float32, device=dev) if want_depth else None,
            "normal": torch.empty((self.total_pixels, 3), dtype=torch.float32, device=dev) if want_normal else None,
        }

    def alloc_labels(self, want_score: bool = True) -> dict:
        dev = self.device
        return {
            "label": torch.empty(self.total_pixels, dtype=torch.int32, device=dev),
            "score": torch.empty(self.total_pixels, dtype=torch.float32, device=dev) if want_score else None,
            "T": torch.empty(self.total_pixels, dtype=torch.float32, device=dev),
            "n": torch.empty(self.total_pixels, dtype=torch.int32, device=dev),
        }

    def render_backward(self, means, scales, quats, opacity, feats, frame: Frame, grad_feat: torch.Tensor):
        """Gradients of sum(grad_feat * frame.feat); returns a dict of tensors.

        The backward reads the records, sorted pairs and tile ranges this
        rasterizer holds, so ``frame`` must be the last frame it rendered;
        otherwise a RuntimeError is raised (render the frame again first)."""
        if frame.generation != self.generation:
            raise RuntimeError(f"render_backward: the frame was rendered from generation {frame.generation} of "
                               f"this rasterizer's lists, which now hold generation {self.generation}; render it "
                               "again before its backward")
        n, C = feats.shape
        dev = self.device
        b = self._bufs
        g = {
            "means": torch.zeros((n, 3), dtype=torch.float32, device=dev),
            "scales": torch.zeros((n, 2), dtype=torch.float32, device=dev),
            "quats": torch.zeros((n, 4), dtype=torch.float32, device=dev),
            "opacity": torch.zeros(n, dtype=torch.float32, device=dev),
            "feats": torch.zeros((n, C), dtype=torch.float32, device=dev),
        }
        grec = torch.empty(self.num_views * n * L.FS_GRAD_RECORD_FLOATS, dtype=torch.float32, device=dev)
        gf = grad_feat.contiguous().float()
        L.check(self.lib.fs_render_backward(_p(means), _p(scales), _p(quats), _p(opacity), _p(b["records"]),
                                            _p(b["vals"]), _p(b["ranges"]), _p(feats), C, n, _p(self.cams_dev),
                                            self.num_views, self.total_tiles, ctypes.byref(self.opts), _p(frame.T),
                                            _p(frame.n), _p(frame.last), _p(gf), _p(grec), _p(g["means"]),
                                            _p(g["scales"]), _p(g["quats"]), _p(g["opacity"]), _p(g["feats"]),
                                            _p(b["ws"]), _stream(dev)), "fs_render_backward")
        return g


def scene_tensors(scene, device="cuda", feat_dtype: str = "f32"):
    """Upload a scene (numpy arrays) as contiguous device tensors."""
    t = lambda a: torch.from_numpy(a).to(device).contiguous()
    feats = t(scene.feats)
    if feat_dtype == "bf16":
        feats = feats.to(torch.bfloat16).contiguous()
    return t(scene.means), t(scene.scales), t(scene.quats), t(scene.opacity), feats


class FrameGraph:
    """One whole frame (preprocess -> bin -> sort -> render) captured as a HIP
    graph and replayed.  The pair count stays on the device (no host
    synchronisation inside the frame); launches are sized by the pair
    capacity established by an eager frame first.  Camera poses can change
    between replays through ``Rasterizer.set_cameras``."""

    def __init__(self, rast: Rasterizer, tensors, *, want_last: bool = False, headroom: float = 1.25):
        self.rast = rast
        self.tensors = tensors
        frame = rast.render(*tensors)                      # sizes the buffers
        need = int(frame.num_pairs * headroom) + 4096
        if need > rast.capacity:
            rast._ensure(tensors[0].shape[0], need)
            rast.render(*tensors)
        self.out = rast.alloc_out(tensors[4].shape[1], want_last=want_last)
        # warm up on a side stream (first launches may initialise the runtime)
        s = torch.cuda.Stream(device=rast.device)
        s.wait_stream(torch.cuda.current_stream(rast.device))
        with torch.cuda.stream(s):
            rast.render_nosync(*tensors, self.out)
        torch.cuda.current_stream(rast.device).wait_stream(s)
        torch.cuda.synchronize(rast.device)
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            rast.render_nosync(*tensors, self.out)
        torch.cuda.synchronize(rast.device)

    def replay(self) -> dict:
        self.rast.generation += 1     # the replay refills the rasterizer's lists
        self.graph.replay()
        return self.out

    def pairs_fit(self) -> bool:
        return self.rast.pairs_fit()


def instance_labels(ins_feats: torch.Tensor, means: torch.Tensor, query_feats: torch.Tensor,
                    query_means: torch.Tensor, query_covs: torch.Tensor, out: torch.Tensor | None = None):
    """Per-Gaussian instance labels, n x Q float32 (softmax over the queries of
    feature similarity x spatial proximity), computed by fs_instance_labels."""
    n, dim = ins_feats.shape
    Q = query_feats.shape[0]
    _f32(ins_feats, (n, dim), "ins_feats")
    _f32(means, (n, 3), "means")
    _f32(query_feats, (Q, dim), "query_feats")
    _f32(query_means, (Q, 3), "query_means")
    _f32(query_covs, (Q, 6), "query_covs")
    lib = L.load()
    if out is None:
        out = torch.empty((n, Q), dtype=torch.float32, device=ins_feats.device)
    L.check(lib.fs_instance_labels(_p(ins_feats), dim, _p(means), n, _p(query_feats), _p(query_means),
                                   _p(query_covs), Q, _p(out), _stream(ins_feats.device)), "fs_instance_labels")
    return out
