"""MI355X-native multi-camera depth ray casting (librc) and its Python binding."""
from .rc import (Scene, Post, Batch, Graph, Server, post_params, downsample, cam_rand, sah_build_host, lib, check, RcError, CAM_DESC,
                 RC_DEPTH_PLANAR, RC_DEPTH_RANGE, RC_POST_NOISE, RC_POST_DROPOUT, RC_POST_LATENCY, RC_POST_SIDEMASK,
                 EXPORTED)

__all__ = ["Scene", "Post", "Batch", "Graph", "Server", "CAM_DESC", "post_params", "downsample", "cam_rand", "sah_build_host", "lib", "check", "RcError", "RC_DEPTH_PLANAR",
           "RC_DEPTH_RANGE", "RC_POST_NOISE", "RC_POST_DROPOUT", "RC_POST_LATENCY", "RC_POST_SIDEMASK", "EXPORTED"]
