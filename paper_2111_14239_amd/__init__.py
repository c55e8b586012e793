"""MI355X-native rounded-KLT block codec (placeholder; the binding is added with the library)."""
