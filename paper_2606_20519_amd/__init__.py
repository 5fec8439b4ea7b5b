"""MI355X-native PSD-cone projection (placeholder; binding added with the C ABI)."""
