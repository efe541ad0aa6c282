"""MI355X-native molecular-dynamics hot path (LJ / Kob-Andersen, Verlet lists,
double-single velocity Verlet) behind the C ABI of libmdx.so."""
from .mdx import (MD_DS, MD_FP32, MD_FP64, MD_MIXED64, PRECISIONS, MdError, MdSystem,  # noqa: F401
                  load, make_config, md_init, md_validate, md_workspace_bytes)
