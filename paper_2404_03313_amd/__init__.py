"""MI355X-native S3TTV / P-PDS hyperspectral denoising and destriping (arXiv 2404.03313)."""
