"""MI355X-native tile-wise LISI / augLISI image similarity (gfx950 HIP).

The compute path is the C-ABI library ``libiqa_hip.so`` (include/iqa.h);
this package only marshals torch tensors into it.
"""

from .iqa import (C_DEFAULT, IqaError, TileResult, auglisi_tiles, check_cfg,  # noqa: F401
                  default_D, default_cfg, iqa_tiles, lisi_tiles, merge_tiles, prepare, pyramid)

__all__ = ["iqa_tiles", "lisi_tiles", "auglisi_tiles", "merge_tiles", "pyramid",
           "default_cfg", "check_cfg", "prepare", "default_D", "C_DEFAULT", "IqaError",
           "TileResult"]
